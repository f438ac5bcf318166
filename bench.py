"""Benchmark: edge-matrix AMG-PCG on one MI355X.

Headline workload: 3D linear elasticity on the unit cube with 128^3 vertices (6,291,456 dofs,
6,242,304 free), P1 Kuhn tetrahedra, E = 1, nu = 0.45, clamped at x = 0, RHS uniform[-1, 1] from
seed 3; two matching passes per level, coarsening until a level has fewer than 500 dofs, one
symmetric multicolour block Gauss-Seidel sweep pre / post; the V-cycle in FP32 (matrices,
vectors and accumulation) inside an FP64 CG (operator, vectors, inner products, stopping test)
to ||r|| <= 1e-8 ||b||.  The V-cycle below the first level of at most 16384 dofs is applied as
its dense matrix (computed at setup from the same hierarchy; the coarsest level is still the
< 500-dof one); that matrix, which holds the coarsest inverse, is read in FP64 with FP64 sums,
as the coarsest inverse is without a tail (--tail-fp32: an FP32 copy).  P_s rows keep at most
4 edge-matrix columns and 6 / 4 real-matrix columns (level 0 / coarser), and the matching
accepts agglomerates whose two-grid bound is below sigma = 18: free parameters (the paper's runs
use caps 4 and 8 / 6 and give no sigma), chosen by measurement for this workload and used for
the 64^3 cube as well; the multi-mesh and learned-coarsening workloads use caps 3 and 6 / 4 with
sigma = 20, measured best there.

A step is one PCG solve to 1e-8, with b resident in HBM when the timed region starts.  Setup
(host coarsening + device P_s / Galerkin / D^+ / coarsest inverse / dense tail) is timed
separately, with its phases split into host, device and copies.  Reported beside the headline
in the same line:
  fp64_vcycle        the same solve with the FP64 V-cycle, and the FP32 solution's distance to it
  sparse_tail        the same hierarchy with every level's sweeps run sparse (no dense tail)
  tail_precision     the same solve with the dense tail read in the other precision
  paper_caps         the same solve with the paper's P_s row caps
  cube64             64^3, nu = 0.3, RHS seed 1, FP64 and FP32 V-cycle; its 32 seeded load
                     cases as one block-panel solve ("batched")
  multi_mesh         16 cubes of 8^3..48^3 vertices, nu uniform in [0.2, 0.45], solved together
  learned_coarsening 96^3 with 200 stiff spherical inclusions: exact against learned walk,
                     with the condition number estimated from the PCG coefficients
  cpu_baseline       the CPU oracle and the GPU on the same 17^3 cube (nu = 0.3, seed 0)

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="vertices per cube side of the headline")
    ap.add_argument("--nu", type=float, default=0.45)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--coarsest", type=int, default=500,
                    help="coarsening stops once a level has fewer dofs than this")
    ap.add_argument("--dense-tail", type=int, default=16384,
                    help="dofs of the largest level whose V-cycle is applied as a dense matrix (0: none)")
    ap.add_argument("--tail-fp32", action="store_true",
                    help="the FP32 V-cycle reads an FP32 copy of the dense tail (default: the FP64 "
                         "tail, which holds the coarsest inverse, with FP64 sums)")
    ap.add_argument("--caps", default="6,4,4",
                    help="headline P_s row caps: real-matrix rows on level 0, on coarser levels, "
                         "edge-matrix rows")
    ap.add_argument("--sigma", type=float, default=18.0,
                    help="headline matching threshold sigma (the two-grid bound of every agglomerate)")
    ap.add_argument("--sub-caps", default="6,4,3",
                    help="P_s row caps of the multi-mesh and learned-coarsening workloads (the 64^3 "
                         "cube uses the headline's)")
    ap.add_argument("--sub-sigma", type=float, default=20.0,
                    help="sigma of the multi-mesh and learned-coarsening workloads")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline solve (for profiler runs)")
    ap.add_argument("--sections", default="all",
                    help="sub-records after the headline: all, or a comma list of sparse_tail, "
                         "tail_precision, paper_caps, cube64, multi, learned, cpu")
    ap.add_argument("--per-colour", action="store_true",
                    help="per-colour records of the FP32 colour sweeps (events around every colour "
                         "launch), also with --headline-only")
    ap.add_argument("--per-level", action="store_true",
                    help="per-level kernel records of both V-cycle precisions, also with --headline-only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=32,
                    help="right-hand sides of the batched block-panel solve at 64^3 (0: skip)")
    ap.add_argument("--multi", type=int, default=16,
                    help="independent meshes of the multi-system solve (0: skip)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-coarsening section")
    ap.add_argument("--learned-n", type=int, default=96)
    ap.add_argument("--learned-inclusions", type=int, default=200)
    ap.add_argument("--counter-pass", action="store_true",
                    help="run only the workload of the rocprofv3 counter passes (no JSON line)")
    return ap.parse_args()


def _progress(msg):
    """One progress line on stderr per finished section (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _caps(spec):
    l0, std, aux = (int(v) for v in spec.split(","))
    return dict(cap_std_l0=l0, cap_std=std, cap_aux=aux)


def _params(E, args, **kw):
    """Setup parameters of the headline."""
    prm = dict(vcycle_fp32=1, coarsest_max_dofs=args.coarsest, dense_tail_dofs=args.dense_tail,
               dense_tail_fp32=int(args.tail_fp32), sigma=args.sigma, **_caps(args.caps))
    prm.update(kw)
    return E.eamg_default_setup_params(**prm)


def _sub_params(E, args, **kw):
    """Setup parameters of the other workloads (their own measured best caps and sigma)."""
    prm = dict(vcycle_fp32=1, coarsest_max_dofs=args.coarsest, dense_tail_dofs=args.dense_tail,
               dense_tail_fp32=int(args.tail_fp32), sigma=args.sub_sigma, **_caps(args.sub_caps))
    prm.update(kw)
    return E.eamg_default_setup_params(**prm)


def _setup(E, torch, p, prm, stream=None):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet, prm, stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    ph = E.eamg_setup_phases(h.h)
    split = {w: round(sum(s for _, s, ww in ph if ww == w), 3) for w in ("host", "device", "copy")}
    return h, {"setup_s": round(setup_s, 3), "split_s": split,
               "phases_s": {n: round(s, 3) for n, s, _ in ph}}


def _timed_solves(E, torch, hier, b, x, stream, steps, warmup, precond):
    for _ in range(warmup):
        hier.solve(b, x, precond=precond, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    infos = []
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        _, info = hier.solve(b, x, precond=precond, stream=stream)
        infos.append(info)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    assert infos[-1]["status"] == E.EAMG_OK and infos[-1]["rel_res_true"] <= 1e-8, infos[-1]
    return ms, infos[-1]


def _kappa(E, h):
    """Condition number of the preconditioned operator estimated by Lanczos from the last
    solve's CG coefficients: T_jj = 1/alpha_j + beta_j/alpha_{j-1}, T_{j,j+1} =
    sqrt(beta_{j+1})/alpha_j; and the CG error reduction factor it implies per iteration."""
    al, be = E.eamg_solve_coefficients(h.h)
    k = len(al)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / al[j] + (be[j] / al[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(be[j + 1]) / al[j]
    ev = np.linalg.eigvalsh(T)
    kap = float(ev[-1] / ev[0])
    return {"kappa": round(kap, 3), "lambda_min": float(ev[0]), "lambda_max": float(ev[-1]),
            "cg_factor": round((np.sqrt(kap) - 1.0) / (np.sqrt(kap) + 1.0), 4)}


# CG kernels of the iteration (everything else the profiler records is the preconditioner)
_CG_KERNELS = ("k_spmv", "k_dot", "k_reduce", "k_update_xr", "k_update_p")


def _profiled(E, hier, b, x, steps, precond, stream):
    """Per-kernel durations with events on the solve stream, over `steps` profiled solves:
    the dominant kernel's roofline and the V-cycle aggregate (algorithmic bytes of all
    preconditioner kernels over their summed durations)."""
    E.eamg_profile_enable(hier.h, True)
    for _ in range(steps):
        hier.solve(b, x, precond=precond, stream=stream)
    kstats = E.eamg_profile_read(hier.h)
    E.eamg_profile_enable(hier.h, False)
    dom = kstats[0]
    achieved = dom["bytes"] / (dom["total_ms"] / 1e3) / 1e9
    roof = {"bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": 8000.0,
            "unit": "GB/s", "frac": achieved / 8000.0, "traffic": _traffic(dom["name"]),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "avg_launch_us": dom["total_ms"] / dom["launches"] * 1e3,
            "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"]}
    vk = [k for k in kstats if not k["name"].startswith(_CG_KERNELS)]
    vb, vt = sum(k["bytes"] for k in vk), sum(k["total_ms"] for k in vk)
    vagg = {"GBps": vb / (vt / 1e3) / 1e9, "frac": vb / (vt / 1e3) / 8e12,
            "ms_per_solve": vt / steps, "bytes_per_solve": vb / steps}
    kern = [{"name": k["name"], "launches_per_step": k["launches"] / steps,
             "ms_per_step": k["total_ms"] / steps,
             "GBps": k["bytes"] / (k["total_ms"] / 1e3) / 1e9 if k["total_ms"] else None}
            for k in kstats[:12]]
    return roof, vagg, kern


def _per_level(E, hier, b, x, precond, stream):
    """Milliseconds per solve of every V-cycle kernel on every level (one profiled solve)."""
    E.eamg_profile_enable(hier.h, 2)
    hier.solve(b, x, precond=precond, stream=stream)
    ks = E.eamg_profile_read(hier.h, 256)
    E.eamg_profile_enable(hier.h, False)
    return [{"name": k["name"], "launches": k["launches"], "ms": round(k["total_ms"], 3),
             "us_per_launch": round(k["total_ms"] / k["launches"] * 1e3, 2),
             "GBps": round(k["bytes"] / (k["total_ms"] / 1e3) / 1e9, 1) if k["total_ms"] else None}
            for k in ks[:40]]


def _per_colour(E, hier, b, x, precond, stream):
    """Time and algorithmic bytes of every colour launch of the sweeps (one profiled solve with
    events around each colour launch, which adds their own dispatch to every launch)."""
    import re
    E.eamg_profile_enable(hier.h, 3)
    hier.solve(b, x, precond=precond, stream=stream)
    ks = E.eamg_profile_read(hier.h, 4096)
    E.eamg_profile_enable(hier.h, False)
    out = []
    for k in ks:
        m = re.match(r"L(\d+) c(\d+) k_gs_color<\w+, (\d+), (true|false)>", k["name"])
        if m:
            out.append({"level": int(m.group(1)), "sweep": "fwd" if m.group(4) == "true" else "bwd",
                        "colour": int(m.group(2)),
                        "us_per_launch": round(k["total_ms"] / k["launches"] * 1e3, 2),
                        "MB_per_launch": round(k["bytes"] / k["launches"] / 1e6, 4)})
    out.sort(key=lambda r: (r["level"], r["sweep"], r["colour"]))
    return out


def _levels(E, h):
    st = h.stats()
    out = []
    for l in range(st["n_levels"]):
        li = E.eamg_level_info_get(h.h, l)
        out.append({"n": li["n"], "bs": li["bs"], "nnzb": li["nnzb_A"], "colors": li["n_colors"],
                    "nnzb_P": li["nnzb_P"]})
    return st, out


def _batch_rhs(p, m):
    """m seeded load cases (case c from default_rng([4, c])), uniform[-1, 1], Dirichlet dofs 0."""
    B = np.stack([np.random.default_rng([4, c]).uniform(-1.0, 1.0, p.n_dofs) for c in range(m)])
    B[:, np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    return B


def _batched(E, torch, hier, p, m, steps, warmup, single_ms):
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
                    "speedup_per_rhs_vs_single_fp64": single_ms * m / ms,
                    "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": ach,
                                 "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                                 "avg_launch_us": dom["total_ms"] / dom["launches"] * 1e3},
                    "kernels": [{"name": k["name"], "launches_per_solve": k["launches"],
                                 "ms_per_solve": k["total_ms"],
                                 "GBps": k["bytes"] / (k["total_ms"] / 1e3) / 1e9}
                                for k in ks[:6]]}
    return out


def _cube64(E, torch, args, stream):
    """64^3, nu = 0.3, RHS seed 1: FP64 V-cycle (the plain FP64 hierarchy and V-cycle) and FP32
    V-cycle, then the batched panel solve of its load cases."""
    from gen import make_problem
    p = make_problem(64, seed=1)
    h, su = _setup(E, torch, p, _params(E, args), stream)
    E.eamg_autotune(h.h, panel_width=max(args.batch, 0), stream=stream)
    b = torch.tensor(p.b, device="cuda")
    x = torch.zeros_like(b)
    out = {"workload": f"elasticity cube 64^3 vertices (786,432 dofs), nu=0.3, RHS seed 1, P_s row caps "
                       f"{args.caps}, sigma {args.sigma:g}",
           "free_dofs": p.n_free_dofs, **su}
    for prec, key in ((E.EAMG_PRECOND_VCYCLE, "fp64_vcycle"), (E.EAMG_PRECOND_VCYCLE_FP32, "fp32_vcycle")):
        ms, info = _timed_solves(E, torch, h, b, x, stream, args.steps, args.warmup, prec)
        out[key] = {"ms_per_solve": ms, "value": p.n_free_dofs / (ms / 1e3), "unit": "dofs/s",
                    "iterations": info["iterations"], "rel_res_true": info["rel_res_true"]}
        # the dominant kernel and the V-cycle aggregate of one profiled solve, as for the
        # headline (the committed counter passes are the headline's: no traffic figure here)
        roof, vagg, _ = _profiled(E, h, b, torch.zeros_like(b), 1, prec, stream)
        out[key]["dominant"] = {k: roof[k] for k in ("kernel", "avg_launch_us", "achieved", "frac",
                                                     "algorithmic_bytes_per_launch")}
        out[key]["vcycle_aggregate"] = {"GBps": vagg["GBps"], "frac": vagg["frac"]}
    out["fp32_speedup_vs_fp64"] = out["fp64_vcycle"]["ms_per_solve"] / out["fp32_vcycle"]["ms_per_solve"]
    st, lv = _levels(E, h)
    out.update({"levels": st["n_levels"], "level_vertices": st["n"], "oc": round(st["oc"], 4),
                "dense_tail": E.eamg_dense_tail(h.h)})
    if args.batch > 0:
        out["batched"] = _batched(E, torch, h, p, args.batch, args.steps, args.warmup,
                                  out["fp64_vcycle"]["ms_per_solve"])
    h.close()
    return out


def _multi_mesh(E, torch, args, count=16, seed=4):
    """Independent meshes of uneven size solved together: count cubes with sides uniform in
    [8, 48] and Poisson ratios uniform in [0.2, 0.45], FP32 V-cycle in FP64 CG, each with its own
    hierarchy; one after another, with eamg_solve_multi (each system's iteration graph on one of
    four streams) and fused into one block-diagonal hierarchy (eamg_fuse, eamg_solve_fused)."""
    from gen import make_problem
    rng = np.random.default_rng(seed)
    sides = rng.integers(8, 49, size=count)
    nus = rng.uniform(0.2, 0.45, size=count)
    t0 = time.perf_counter()
    sysm = []
    for c, (n, nu) in enumerate(zip(sides, nus)):
        p = make_problem(int(n), nu=float(nu), seed=100 + c)
        h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                        _sub_params(E, args))
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
    for _ in range(args.steps):
        for (p, h), b, x in zip(sysm, bs, xs):
            h.solve(b, x, precond=prec)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    E.eamg_solve_multi(hs, bs, xs, precond=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, infos = E.eamg_solve_multi(hs, bs, xs, precond=prec)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    assert st == E.EAMG_OK and max(i["rel_res_true"] for i in infos) <= 1e-8
    dofs = sum(p.n_free_dofs for p, _ in sysm)
    out = {"meshes": [int(n) for n in sides], "free_dofs": dofs, "setup_s": round(setup_s, 3),
           "dtype": "f32 V-cycle in f64 CG", "ms_one_after_another": seq_ms,
           "streams": {"ms_per_solve_all": ms, "value": dofs / (ms / 1e3), "unit": "dofs/s",
                       "speedup_vs_one_after_another": seq_ms / ms,
                       "iterations": [i["iterations"] for i in infos]}}
    # one block-diagonal hierarchy for all systems (eamg_fuse): V-cycles ending at dense tails of
    # at most 4096 dofs built for the fused hierarchy, at every coarsest inverse, and at the
    # systems' own tails (<= 16384 dofs)
    for key, tails in (("fused", 4096), ("fused_no_tails", 0), ("fused_own_tails", -1)):
        t0 = time.perf_counter()
        f = E.Fused([h for _, h in sysm], dense_tail_dofs=tails)
        fuse_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        E.eamg_autotune(f.h, 0)
        tune_s = time.perf_counter() - t0
        f.solve(bs, xs, precond=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, st, finfo = f.solve(bs, xs, precond=prec)
        torch.cuda.synchronize()
        fms = (time.perf_counter() - t0) * 1e3 / args.steps
        assert st == E.EAMG_OK and max(i["rel_res_true"] for i in finfo) <= 1e-8
        f.close()
        out[key] = {"dense_tail_dofs": tails, "ms_per_solve_all": fms,
                    "value": dofs / (fms / 1e3), "unit": "dofs/s",
                    "fuse_s": round(fuse_s, 3), "autotune_s": round(tune_s, 3),
                    "speedup_vs_one_after_another": seq_ms / fms, "speedup_vs_streams": ms / fms,
                    "iterations": [i["iterations"] for i in finfo],
                    "max_rel_res_true": max(i["rel_res_true"] for i in finfo)}
    for _, h in sysm:
        h.close()
    best = min(out["streams"]["ms_per_solve_all"], out["fused"]["ms_per_solve_all"])
    out.update({"ms_per_solve_all": best, "value": dofs / (best / 1e3), "unit": "dofs/s",
                "speedup_vs_one_after_another": seq_ms / best})
    return out


def _learned(E, torch, args, stream):
    """Learned coarsening on a heterogeneous cube (stiff spherical inclusions, E = 1e4, nu of each
    inclusion uniform in [0.3, 0.49]): the edge network is trained on the GPU on small meshes of
    the same kind (their exact criterion decisions), then the exact and the learned walk build
    hierarchies of the large mesh; criteria evaluations, setup time, PCG iterations, and the
    condition number of the preconditioned operator (Lanczos from the PCG coefficients) are
    compared."""
    from gen import make_problem
    n, inclusions = args.learned_n, args.learned_inclusions

    t0 = time.perf_counter()
    graphs = []
    for c, (m, inc, nu) in enumerate([(12, 8, 0.3), (14, 12, 0.4), (16, 16, 0.35), (13, 10, 0.45)]):
        p = make_problem(m, inclusions=inc, nu=nu, geometry_seed=10 + c, seed=c)
        h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                        E.eamg_default_setup_params(gnn_record=1))
        for k in range(E.eamg_coarsening_stats(h.h)["sample_passes"]):
            X, edges, nn, y, w = E.eamg_gnn_samples(h.h, k)
            if len(y) and w.sum() > 0:
                graphs.append((X, edges, nn, y, w))
        h.close()
    net = E.EdgeNet(seed=3)
    hist = net.train(graphs, epochs=200, lr=3e-3)
    train_s = time.perf_counter() - t0
    p = make_problem(n, inclusions=inclusions, nu=0.3, geometry_seed=5, seed=5)
    b = torch.tensor(p.b, device="cuda")
    out = {"workload": f"elasticity cube {n}^3, {inclusions} stiff spherical inclusions (E=1e4, "
                       f"nu uniform [0.3, 0.49]) in E=1, nu=0.3, RHS seed 5; network trained on "
                       f"4 meshes of 12^3..16^3",
           "train_s": round(train_s, 3), "train_loss": [float(hist[0]), float(hist[-1])]}
    for key, kw in (("exact", {}), ("learned", {"gnn": net.h.value, "gnn_skip": 0.2})):
        h, su = _setup(E, torch, p, _sub_params(E, args, **kw), stream)
        st = E.eamg_coarsening_stats(h.h)
        x, info = h.solve(b, precond=E.EAMG_PRECOND_VCYCLE_FP32, stream=stream)
        kap = _kappa(E, h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.solve(b, x, precond=E.EAMG_PRECOND_VCYCLE_FP32, stream=stream)
        torch.cuda.synchronize()
        out[key] = {**su, "criteria_evaluations": st["evaluated"],
                    "mu_g_evaluations": st["evaluated_g"], "passed_over": st["skipped"],
                    "pcg_iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                    "solve_ms": round((time.perf_counter() - t0) * 1e3, 2),
                    "oc": round(h.stats()["oc"], 4), **kap}
        h.close()
    net.close()
    out["evaluations_saved"] = 1.0 - out["learned"]["criteria_evaluations"] / out["exact"]["criteria_evaluations"]
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(E, torch, args, stream):
    """The CPU oracle (FP64 NumPy/SciPy, one process, BLAS held to one thread) and the GPU on the
    same bounded sample: the 17^3-vertex cube (14,739 dofs), nu = 0.3, RHS seed 0, PCG to 1e-8;
    the oracle's solve (median of 3) and setup are timed, and beside it the library's FP64 solve
    of the same problem with the oracle's settings and with the headline's."""
    from threadpoolctl import threadpool_limits

    import oracle
    from gen import make_problem
    p = make_problem(17, seed=0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
        t_setup = time.perf_counter() - t0
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            xo, it, rel, rel_true, conv = oracle.pcg(ho, p.b, rtol=1e-8)
            times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    b = torch.tensor(p.b, device="cuda")
    gpu = {}
    # the oracle's own settings (default setup parameters: the same hierarchy, so the same
    # iterations), then the headline's
    for key, prm in (("gpu_same_input", E.eamg_default_setup_params()),
                     ("gpu_headline_settings", _params(E, args))):
        h, su = _setup(E, torch, p, prm, stream)
        x = torch.zeros_like(b)
        gms, ginfo = _timed_solves(E, torch, h, b, x, stream, max(args.steps, 5), 1,
                                   E.EAMG_PRECOND_VCYCLE)
        err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
        h.close()
        gpu[key] = {"dtype": "f64", "ms_per_solve": gms, "value": p.n_free_dofs / (gms / 1e3),
                    "iterations": ginfo["iterations"], "rel_res_true": ginfo["rel_res_true"],
                    "setup_s": su["setup_s"], "x_rel_diff_vs_oracle": err}
    return {"value": p.n_free_dofs / t, "unit": "dofs/s", "cores": 1, "kind": "oracle",
            "sample": f"17^3-vertex cube ({p.n_free_dofs} free dofs), nu=0.3, RHS seed 0: oracle "
                      f"setup {t_setup:.1f} s, PCG to 1e-8 in {it} iterations, median of 3 solves "
                      f"{t:.3f} s, one thread (the 64^3 and 128^3 oracle setups would take "
                      f"minutes to hours and are not run)",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "oracle_setup_s": round(t_setup, 2), "oracle_solve_s": round(t, 4),
            "oracle_iterations": it, **gpu,
            "gpu_speedup_solve": t * 1e3 / gpu["gpu_same_input"]["ms_per_solve"]}


def _traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None if
    the summary is for another kernel or kernels.hip has changed since it was measured."""
    import hashlib
    import re
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        txt = open(os.path.join(root, "profiles", "traffic_k_gs_color_cube128.md")).read()
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


def _counter_pass(args):
    """Workload of the rocprofv3 counter passes: a calibration copy of 64 MiB, then one solve of
    the headline problem (FP32 V-cycle) with eager launches.  Prints the launches of every kernel
    in that solve (the last dispatches of each kernel in the counter output are the solve's)."""
    os.environ["EAMG_GRAPH"] = "0"
    import torch
    import paper_2011_13325_amd as E
    from gen import make_problem
    torch.cuda.set_device(0)
    n = 8 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    p = make_problem(args.n, nu=args.nu, seed=args.seed)
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet, _params(E, args))
    E.eamg_autotune(h.h, 0)
    E.eamg_profile_enable(h.h, True)
    x, info = h.solve(torch.tensor(p.b, device="cuda"), precond=E.EAMG_PRECOND_VCYCLE_FP32)
    torch.cuda.synchronize()
    ks = E.eamg_profile_read(h.h)
    E.eamg_profile_enable(h.h, False)
    print(f"counter pass: copy of {8 * n} bytes; solve {info['iterations']} iterations", flush=True)
    print("solve launches: " + json.dumps({k["name"]: {"launches": k["launches"], "bytes": k["bytes"]}
                                           for k in ks}), flush=True)
    h.close()


def main():
    args = _args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.counter_pass:
        _counter_pass(args)
        return
    import torch
    import paper_2011_13325_amd as E
    from gen import make_problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    p = make_problem(args.n, nu=args.nu, seed=args.seed)
    hier, su = _setup(E, torch, p, _params(E, args), stream)
    _progress(f"headline setup {su['setup_s']} s")
    t0 = time.perf_counter()
    tune_before, tune_after = E.eamg_autotune(hier.h, panel_width=0, stream=stream)
    tune_s = time.perf_counter() - t0
    st, level_info = _levels(E, hier)
    b = torch.tensor(p.b, device=dev)
    x32 = torch.zeros_like(b)
    P32, P64 = E.EAMG_PRECOND_VCYCLE_FP32, E.EAMG_PRECOND_VCYCLE
    ms, info = _timed_solves(E, torch, hier, b, x32, stream, args.steps, args.warmup, P32)
    kap32 = _kappa(E, hier)
    _progress(f"headline FP32 solve {ms:.3f} ms, {info['iterations']} iterations")
    roof, vagg, kern = _profiled(E, hier, b, torch.zeros_like(b), args.steps, P32, stream)
    x64 = torch.zeros_like(b)
    ms64, info64 = _timed_solves(E, torch, hier, b, x64, stream, args.steps, args.warmup, P64)
    kap64 = _kappa(E, hier)
    _, vagg64, kern64 = _profiled(E, hier, b, torch.zeros_like(b), 1, P64, stream)
    xdiff = float((x32 - x64).norm() / x64.norm())
    _progress(f"headline FP64 solve {ms64:.3f} ms")
    vbytes, itbytes = E.eamg_traffic_model(hier.h, P32)
    vbytes64, itbytes64 = E.eamg_traffic_model(hier.h, P64)
    its = info["iterations"]
    value = p.n_free_dofs / (ms / 1e3)
    tail = E.eamg_dense_tail(hier.h)
    out = {
        "metric": "AMG-PCG time to 1e-8 and dofs/s, FP64 vs mixed/batched; V-cycle HBM GB/s",
        "value": value, "unit": "dofs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"elasticity cube {args.n}^3 vertices ({p.n_dofs} dofs; Kuhn P1, "
                               f"E=1, nu={args.nu}, clamped x=0, RHS seed {args.seed}), FP32 "
                               f"V-cycle in FP64 CG to 1e-8, coarsening to < {args.coarsest} "
                               f"dofs, dense V-cycle tail <= {args.dense_tail} dofs, P_s row caps "
                               f"{args.caps}, sigma {args.sigma:g}",
                   "p_s_caps": _caps(args.caps), "sigma": args.sigma,
                   "multi_mesh_and_learned": {"p_s_caps": _caps(args.sub_caps), "sigma": args.sub_sigma},
                   "precision": "V-cycle FP32 (matrices, vectors, accumulation; the dense tail "
                                "with the coarsest inverse " +
                                ("FP32 with FP64 sums" if args.tail_fp32 else "FP64") + "); CG FP64",
                   "coarsest_max_dofs": args.coarsest, "dense_tail": {"level": tail[0], "dofs": tail[1]},
                   "dofs": p.n_dofs, "free_dofs": p.n_free_dofs, "iterations": its,
                   "rel_res_true": info["rel_res_true"], "levels": st["n_levels"],
                   "level_vertices": st["n"], "vc": round(st["vc"], 4), "oc": round(st["oc"], 4),
                   "setup": su,
                   "autotune": {"s": round(tune_s, 3), "tuned_ms_before": tune_before,
                                "tuned_ms_after": tune_after},
                   "model_bytes_per_iteration": itbytes,
                   "model_GBps_whole_solve": itbytes * its / (ms / 1e3) / 1e9,
                   "level_info": level_info},
    }
    out["roofline"] = roof
    out["vcycle_aggregate"] = vagg
    out["kappa_estimate"] = kap32
    out["kernels"] = kern
    out["fp64_vcycle"] = {
        "value": p.n_free_dofs / (ms64 / 1e3), "unit": "dofs/s", "ms_per_step": ms64,
        "iterations": info64["iterations"], "rel_res_true": info64["rel_res_true"],
        "fp32_speedup": ms64 / ms, "model_bytes_per_iteration": itbytes64,
        "vcycle_aggregate": vagg64, "kappa_estimate": kap64, "kernels": kern64[:8],
        "fp32_solution_rel_diff": xdiff}
    if not args.headline_only or args.per_level:
        out["per_level_fp32"] = _per_level(E, hier, b, torch.zeros_like(b), P32, stream)
    if args.per_level:
        out["per_level_fp64"] = _per_level(E, hier, b, torch.zeros_like(b), P64, stream)
    if args.per_colour:
        out["per_colour_fp32"] = _per_colour(E, hier, b, torch.zeros_like(b), P32, stream)
    hier.close()

    def want(name):
        return not args.headline_only and (args.sections == "all" or name in args.sections.split(","))

    if not args.headline_only:
        if want("sparse_tail") and args.dense_tail > 0:
            h2, su2 = _setup(E, torch, p, _params(E, args, dense_tail_dofs=0), stream)
            E.eamg_autotune(h2.h, panel_width=0, stream=stream)
            ms2, info2 = _timed_solves(E, torch, h2, b, torch.zeros_like(b), stream, args.steps,
                                       args.warmup, P32)
            out["sparse_tail"] = {"ms_per_step": ms2, "value": p.n_free_dofs / (ms2 / 1e3),
                                  "iterations": info2["iterations"], "setup_s": su2["setup_s"],
                                  "dense_tail_speedup": ms2 / ms}
            h2.close()
            _progress(f"sparse tail {ms2:.3f} ms")
        if want("tail_precision") and args.dense_tail > 0:
            # the same hierarchy with the dense tail read in the other precision
            t32 = 0 if args.tail_fp32 else 1
            h4, su4 = _setup(E, torch, p, _params(E, args, dense_tail_fp32=t32), stream)
            E.eamg_autotune(h4.h, panel_width=0, stream=stream)
            x4 = torch.zeros_like(b)
            ms4, info4 = _timed_solves(E, torch, h4, b, x4, stream, args.steps, args.warmup, P32)
            out["tail_precision"] = {"dense_tail_fp32": t32, "ms_per_step": ms4,
                                     "value": p.n_free_dofs / (ms4 / 1e3),
                                     "iterations": info4["iterations"],
                                     "rel_res_true": info4["rel_res_true"],
                                     "solution_rel_diff_vs_fp64_vcycle": float((x4 - x64).norm() / x64.norm()),
                                     "speedup_vs_headline": ms / ms4}
            h4.close()
            _progress(f"tail precision {ms4:.3f} ms")
        # the paper's P_s row caps (4 for edge-matrix rows, 8 / 6 for real-matrix rows)
        paper = dict(cap_std_l0=8, cap_std=6, cap_aux=4)
        if want("paper_caps") and paper != _caps(args.caps):
            h3, su3 = _setup(E, torch, p, _params(E, args, **paper), stream)
            E.eamg_autotune(h3.h, panel_width=0, stream=stream)
            ms3, info3 = _timed_solves(E, torch, h3, b, torch.zeros_like(b), stream, args.steps,
                                       args.warmup, P32)
            out["paper_caps"] = {"p_s_caps": paper, "ms_per_step": ms3,
                                 "value": p.n_free_dofs / (ms3 / 1e3),
                                 "iterations": info3["iterations"], "oc": round(h3.stats()["oc"], 4),
                                 "setup_s": su3["setup_s"], "tuned_caps_speedup": ms3 / ms}
            h3.close()
            _progress(f"paper caps {ms3:.3f} ms")
        if want("cube64"):
            out["cube64"] = _cube64(E, torch, args, stream)
            _progress("64^3 and batched panel done")
        if want("multi") and args.multi > 0:
            out["multi_mesh"] = _multi_mesh(E, torch, args, count=args.multi)
            _progress("multi-mesh done")
        if want("learned") and not args.no_learned:
            out["learned_coarsening"] = _learned(E, torch, args, stream)
            _progress("learned coarsening done")
        if want("cpu") and not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(E, torch, args, stream)
    E.close_all()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
