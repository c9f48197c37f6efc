"""Benchmark of the PBM + multigrid-MINRES hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Default run: the 192x96x96 cantilever with three point loads (5.4 M DOFs, the
largest single-GPU workload).  A step is one pass of the whole hot path on
it: one outer iteration of Algorithm 1 in mixed precision (evaluation,
gradient and reduced right-hand side, multigrid setup, MINRES preconditioned
by one V-cycle per iteration, Newton completion and Armijo search, multiplier
and penalty update) and K(rho)u in FP64 on a batch of at least 8 independent
(x, y, rho) sets (more than 1 GB, beyond the 256 MB Infinity Cache).  Inputs
are resident on the device before the timed region.

Printed: one JSON line.  value = K(rho)u throughput in GDOF/s over every
launch in the timed region (HIP events on the library's stream), with its
roofline against the compulsory bytes (read x and rho, write y); the hot
path's rates (outer iterations, MINRES-MG iterations per second), MINRES-MG
at a fixed Newton point in FP64 and mixed precision, time-to-KKT of the
64x32x32 cantilever in FP64 and mixed, and the CPU oracle's K(rho)u on the
same workload.  Other modes (--solve, --serve, --doc, --ip, --paper, --scale,
--scale-kernels, --kernels) are listed by --help.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "K(rho)u GDOF/s + MINRES-MG iters/s; time-to-KKT 1e-6 per VTS; p50/p99"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=1,
                    help="--solve / --kernels: 0 cantilever 8x4x4, 1 cantilever 64x32x32, "
                         "2 bridge 128x64x64, 3 cantilever 192x96x96 (three point loads)")
    ap.add_argument("--solve", action="store_true",
                    help="time-to-KKT: complete PBM solves of --workload from the initial "
                         "point, --steps timed after --warmup")
    ap.add_argument("--precision", choices=["config", "fp64", "mixed"], default="config",
                    help="override the workload's precision (mixed: FP32 multigrid)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--kernels", action="store_true",
                    help="kernel-only run for hardware-counter passes: R V-cycles, R K(rho)x, "
                         "R S-applies at the initial Newton point and R plain copies of "
                         "256 MiB (the counter scale reference); prints one JSON line")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--serve", action="store_true",
                    help="serving stream: Poisson arrivals of mixed VTS requests against the "
                         "request loop; prints one JSON line with p50/p99 latency per rate")
    ap.add_argument("--doc", action="store_true",
                    help="the damped optimality-criteria method (the paper's comparison "
                         "method) on the same workload and device: time to its stopping "
                         "test, beside PBM's time-to-KKT; prints one JSON line")
    ap.add_argument("--ip", action="store_true",
                    help="the primal-dual interior point method (the paper's other comparison "
                         "method) on the same workload in FP64, beside PBM; one JSON line")
    ap.add_argument("--paper", action="store_true",
                    help="the paper's CANT/BRIDGE-4-2-2-{5,6} problems with the paper's "
                         "parameters (Section 7), iteration counts beside Tables 3 and 4 "
                         "(with --ip: the interior point method)")
    ap.add_argument("--scale", action="store_true",
                    help="time-to-KKT of the benchmark cantilever family at refinement levels "
                         "--levels (n up to 12.8 M DOFs); one JSON line")
    ap.add_argument("--levels", type=int, nargs="+", default=[5, 6, 7])
    ap.add_argument("--kinds", nargs="+", default=["CANT", "BRIDGE"],
                    choices=["CANT", "BRIDGE"], help="problem kinds (--paper)")
    ap.add_argument("--families", type=int, nargs="+", default=[2, 4, 6, 8],
                    help="m_x of the CANT/BRIDGE-m_x-2-2-l problems (--paper)")
    ap.add_argument("--cap-seconds", type=float, default=600.0,
                    help="wall-time cap of one solve (--paper)")
    ap.add_argument("--paper-only", action="store_true",
                    help="--paper: only the paper's parameters, not the library's")
    ap.add_argument("--library-rho-lo", type=float, default=1e-3,
                    help="--paper: lower bound of rho for the library-option solve")
    ap.add_argument("--multiload", action="store_true",
                    help="several load cases: batched K(rho) on the three point-load cases of "
                         "the 192x96x96 cantilever, the stacked S-apply, V-cycle and MINRES-MG "
                         "there, and time-to-KKT of the two-case 64x32x32 cantilever")
    ap.add_argument("--ml-no-solve", action="store_true",
                    help="--multiload without the time-to-KKT solve (counter passes)")
    ap.add_argument("--scale-kernels", action="store_true",
                    help="the dominant kernels (finest Gauss-Seidel pass, K(rho)x, S-apply) "
                         "timed at each of --levels, FP64 and mixed; one JSON line")
    ap.add_argument("--requests", type=int, default=256, help="requests per rate (--serve)")
    ap.add_argument("--rates", type=float, nargs="+", default=[0.5, 0.8, 1.2],
                    help="--serve: arrival rates as multiples of 1 / mean alone service time")
    ap.add_argument("--t-alone", type=float, default=None,
                    help="--serve: mean alone service time to use (default: measured)")
    ap.add_argument("--burst", type=int, default=None,
                    help="--serve: --requests requests of serving grid index BURST at once, "
                         "batching on and off")
    ap.add_argument("--no-batching", action="store_true",
                    help="--serve: each request's launches on its own stream")
    ap.add_argument("--slots", type=int, default=4, help="concurrent requests (--serve)")
    ap.add_argument("--pool-gb", type=float, default=16.0, help="device pool (--serve)")
    return ap.parse_args()


def kernel_roofline(torch, ctx, pr, reps=200):
    """K(rho)x in FP64 timed with HIP events on the library's stream.
    Algorithmic bytes per launch: read x and write y (8 B x n_dof each), read
    rho (8 B x m) and the DOF mask (1 B x n_dof)."""
    n_dof, m = pr.n_dof, pr.m
    bytes_per = 8 * n_dof * 2 + 8 * m + n_dof
    # rotating buffers so that the working set exceeds the 256 MB Infinity Cache
    per_set = 16 * n_dof
    nsets = max(2, int(math.ceil(512e6 / per_set)))
    xs = [torch.rand(n_dof, dtype=torch.float64, device="cuda") for _ in range(nsets)]
    ys = [torch.empty(n_dof, dtype=torch.float64, device="cuda") for _ in range(nsets)]
    stream = torch.cuda.current_stream()
    for i in range(nsets):
        ctx.apply_K(xs[i], ys[i])
    res = {}
    for label, sets in (("rotating", nsets), ("hot", 1)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            k = i % sets
            ctx.apply_K(xs[k], ys[k])
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[label] = dict(ms=ms, gbs=bytes_per / (ms * 1e-3) / 1e9,
                          gdofs=n_dof / (ms * 1e-3) / 1e9)
    del xs, ys
    return bytes_per, res


def kernel_source_hash():
    """Hash of the multigrid kernels' source and of the level structure they
    read (their counters stay valid while both are unchanged)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1904_06556_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "mg.hip"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "vts_internal.hpp")) as fh:
        hdr = fh.read()
    a = hdr.index("struct Level {")
    h.update(hdr[a:hdr.index("};", a)].encode())
    return h.hexdigest()[:16]


def operator_source_hash():
    """Hash of the operator kernels' source (K(rho)u and the S-apply; their
    counters stay valid while it is unchanged)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1904_06556_amd", "csrc", "operator.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def multiload_source_hash():
    """Hash of the multi-load kernels' source."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1904_06556_amd", "csrc", "multiload.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_file(workload_name):
    return os.path.join(ROOT, "profiles", f"traffic_pmc_{workload_name}.md")


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch of `kernel` on `workload_name` from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (each counter scaled by what it
    reads for a plain copy); None if there is none or if the kernel's source
    changed since the counters were taken."""
    path = traffic_file(workload_name)
    if not os.path.exists(path):
        return None
    val, hashes = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith(f"traffic_bytes_per_launch {kernel} ="):
                val = float(line.split("=")[1])
            elif "_source_sha256_16 =" in line:
                k, v = line.split("=")
                hashes[k.strip()] = v.strip()
    if kernel.startswith("k_ml_"):
        key, now = "multiload_source_sha256_16", multiload_source_hash()
    elif kernel.startswith(("k_apply_K", "k_S_plane")):
        key, now = "operator_source_sha256_16", operator_source_hash()
    else:
        key, now = "kernel_source_sha256_16", kernel_source_hash()
    return val if (val is not None and hashes.get(key) == now) else None


def profiled(ctx, kernel_class, run):
    """Average duration and algorithmic bytes of every launch of one kernel
    class during `run()`, timed by the library with HIP events recorded on
    its own stream around each launch."""
    ctx.profile_start(kernel_class)
    run()
    p = ctx.profile_stop()
    n = max(p["launches"], 1)
    ms = p["total_ms"] / n
    bpl = p["bytes"] / n
    return dict(launches=p["launches"], avg_launch_ms=ms, bytes_per_launch=bpl,
                gbs=bpl / (ms * 1e-3) / 1e9 if ms > 0 else 0.0)


def minres_rate(torch, ctx, its=50):
    """MINRES-MG iterations per second at the converged Newton point (fixed
    iteration count: tolerance 0)."""
    ctx.newton_setup()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.solve_newton(0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return st["iterations"] / dt, st["iterations"]


def cpu_baseline(pr, eps_mr0, newton_steps_gpu, budget_s):
    """The FP64 oracle on the host cores: Newton steps of the same solve from
    the same initial point until `budget_s` is spent; scaled to VTS/s with the
    GPU solve's Newton count."""
    from oracle import pbm as opbm
    opts = opbm.Options(max_newton=1000)
    if eps_mr0:
        opts.eps_mr0 = eps_mr0
    s = opbm.Solver(pr, opts)
    st = opbm.initial_state(s.P.grid.n_dof, s.P.grid.m, s.P.V)
    t0 = time.perf_counter()
    done = 0
    eps = opts.eps_nwt0
    while time.perf_counter() - t0 < budget_s and done < 50:
        s.opts.max_newton = 1
        st, _ = s.newton(st, 0.0)
        done += 1
    dt = time.perf_counter() - t0
    per_newton = dt / max(done, 1)
    vts_per_s = 1.0 / (per_newton * max(newton_steps_gpu, 1))
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return dict(value=vts_per_s, unit="VTS/s", cores=1, cores_available=cores, kind="oracle",
                sample=(f"first {done} Newton steps of the same {pr.name} solve "
                        f"({per_newton:.2f} s each: evaluation, assembled S, Galerkin "
                        f"hierarchy, MINRES-MG, line search), scaled by the GPU solve's "
                        f"{newton_steps_gpu} Newton steps; SciPy sparse kernels run on one "
                        f"thread"),
                seconds_per_newton=per_newton)


def kernels_only(a, torch, W, V):
    """Each hot kernel a fixed number of times, for rocprofv3 counter passes."""
    pr = W.config(a.workload)
    prec = V.VTS_MIXED if pr.extra.get("precision") == "mixed" else V.VTS_FP64
    ctx = V.Context.from_problem(pr, precision=prec)
    ctx.reset()
    ctx.newton_setup()
    g = torch.Generator(device="cpu").manual_seed(1)
    r = (torch.rand(ctx.n_dof + 1, generator=g, dtype=torch.float64) - 0.5).cuda()
    z = torch.empty_like(r)
    # K(rho)x on rotating (x, y, rho) sets beyond the Infinity Cache, as timed
    # by the default run
    k_bytes = 16.0 * ctx.n_dof + 8.0 * ctx.m
    nsets = max(8, int(math.ceil(K_SET_BYTES / k_bytes)))
    xs = [(torch.rand(ctx.n_dof, generator=g, dtype=torch.float64) - 0.5).cuda()
          for _ in range(nsets)]
    rs = [(1e-3 + torch.rand(ctx.m, generator=g, dtype=torch.float64)).cuda()
          for _ in range(nsets)]
    ys = [torch.empty_like(xs[0]) for _ in range(nsets)]
    for _ in range(a.reps):
        ctx.precondition(r, z)
    for q in range(a.reps * nsets):
        ctx.apply_K_rho(rs[q % nsets], xs[q % nsets], ys[q % nsets])
    for _ in range(a.reps):
        ctx.apply_S(r, z)
    copy_bytes = 256 << 20
    src = torch.ones(copy_bytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernels", "workload": pr.name, "reps": a.reps,
                      "k_sets": nsets, "k_launches": a.reps * nsets, "k_bytes": k_bytes,
                      "operator_source_sha256_16": operator_source_hash(),
                      "kernel_source_sha256_16": kernel_source_hash(),
                      "n_dof": ctx.n_dof, "m": ctx.m,
                      "copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes}),
          flush=True)
    ctx.close()
    return 0


def paper_names(a):
    """CANT-mx-2-2-l and BRIDGE-mx-2-2-l for the selected mx and l (Tables 3, 4)."""
    return [f"{kind}-{mx}-2-2-{l}" for kind in a.kinds for l in a.levels
            for mx in a.families]


def paper_problem(W, name):
    kind, mx, my, mz, l = name.split("-")
    gen = W.paper_cantilever if kind == "CANT" else W.paper_bridge
    return gen(int(mx), int(my), int(mz), int(l))


def paper_problems_ip(a, torch, W, V):
    """The interior point method with the paper's parameters (Algorithm 3:
    eps_IP = 1e-5, sigma = 0.2, r = s = 1e-2 initially; rho_lo = 1e-3 as in
    Section 7 for IP) on the selected CANT and BRIDGE problems, FP64."""
    from workloads import paper_tables as T

    def run(pr, name, eps_mr0):
        ctx = V.Context.from_problem(pr, precision=V.VTS_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.ip_init(eps_mr0=eps_mr0)
        its, mr, status, s = 0, 0, V.VTS_ENOTCONV, {}
        for k in range(150):
            s = ctx.ip_step(check=False)
            its, mr = k + 1, mr + s["minres_its"]
            if its % 10 == 0 or s["converged"] or s["status"] != V.VTS_OK:
                print(f"{name} IP (eps_MR0 {eps_mr0:g}): iteration {its} minres "
                      f"{s['minres_its']} gap ratio {s['gap_ratio']:.2e} res_IP "
                      f"{s['res_ip']:.2e} t {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
            if s["status"] != V.VTS_OK:
                status = s["status"]
                break
            if s["converged"]:
                status = V.VTS_OK
                break
            if time.perf_counter() - t0 > a.cap_seconds:
                status = "time cap"
                break
        torch.cuda.synchronize()
        res = dict(seconds=time.perf_counter() - t0,
                   status=status if isinstance(status, str) else int(status),
                   iterations=its, minres=mr, compliance=s.get("compliance"), eps_mr0=eps_mr0)
        ctx.close()
        return res

    out = {}
    for name in paper_names(a):
        pr = paper_problem(W, name)
        pr.rho_lo = 1e-3
        res = dict(m=pr.m, n=pr.n, paper_ip_its_mr=T.entry(name)["ip"])
        res["paper_eps_mr0"] = run(pr, name, 1e-2)
        if res["paper_eps_mr0"]["status"] != V.VTS_OK:
            # the paper's start value leaves the first directions too inexact
            # for this load; the same method with a tighter start
            res["eps_mr0_1e-4"] = run(pr, name, 1e-4)
        out[name] = res
        print(f"{name}: {json.dumps(res)}", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "value": None, "unit": "see problems", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "paper problems (Section 7), interior point method with "
                                   "the paper's parameters"},
            "problems": out}
    print(json.dumps(line), flush=True)
    return 0


def paper_options(V, name, n):
    """PBM with the parameter values stated after Algorithm 1 and in Section 7
    (eps_PBM = 1e-5, eps_NWT_min = 1e-3, final eps_NWT = 10 eps_PBM, absolute
    floors p_min = q_min = 1e-8, eps_MR0 = 1e-4 sqrt(n), no KKT test, u the
    last Newton iterate) and the footnote overrides of Tables 3 and 4."""
    from workloads import paper_tables as T
    o = dict(eps_pbm=1e-5, eps_nwt_min=1e-3, eps_nwt_final=1e-4, final_res4=0, eps_stat=0.0,
             accept_stall=0.0, p_min=1e-8, q_min=1e-8, p_min_relative=0, eps_mr0=0.0,
             max_outer=100, kkt_tol=0.0, eps_state=0.0)
    o.update(T.paper_overrides(name, n))
    return V.default_options(**o), T.paper_overrides(name, n)


def run_pbm_capped(torch, V, ctx, name, label, cap_s, max_outer):
    """Outer PBM iterations one call at a time (progress on stderr), then the
    final Newton call, rho update and KKT evaluation of vts_pbm_solve; stops
    early at cap_s seconds."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, s = V.VTS_OK, {}
    for k in range(max_outer):
        try:
            s = ctx.pbm_iterate()
        except V.VtsError as e:
            status = e.status
            break
        print(f"{name} [{label}]: outer {k + 1} ratio {s['ratio']:.2e} newton "
              f"{s['newton_its']} minres {s['minres_its']} t {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        if s["converged"]:
            break
        if time.perf_counter() - t0 > cap_s:
            status = "time cap"
            break
    r = ctx.pbm_solve(check=False) if status == V.VTS_OK else None
    torch.cuda.synchronize()
    res = dict(seconds=time.perf_counter() - t0,
               status=status if isinstance(status, str) else int(r["status"] if r else status),
               last_gap_ratio=s.get("ratio"))
    if r:
        res.update({k: r[k] for k in ("outer", "newton", "minres", "compliance", "res_pbm",
                                      "kkt", "r_eq", "r_vol", "r_box", "r_stat")})
    else:
        st = ctx.state_dict()
        res.update(outer=int(st["outer"]), newton=int(st["newton"]), minres=int(st["minres"]))
    print(f"{name} [{label}] result: {json.dumps(res)}", file=sys.stderr, flush=True)
    return res


def paper_problems(a, torch, W, V):
    """The CANT-mx-2-2-l and BRIDGE-mx-2-2-l problems of Tables 3 and 4 (the
    selected mx and l): PBM with the paper's parameters and footnote
    overrides (counts beside the tables'), then the same problem with this
    library's options in mixed precision with rho_lo = --library-rho-lo
    (time to KKT <= 1e-6)."""
    from workloads import paper_tables as T
    prec = V.VTS_MIXED if a.precision == "mixed" else V.VTS_FP64
    out = {}
    for name in paper_names(a):
        pr = paper_problem(W, name)
        e = T.entry(name)
        res = dict(m=pr.m, n=pr.n, paper_pbm_outer_nwt_mr=e["pbm"],
                   paper_flags=list(e["flags"]), paper_res_pbm=e["res_pbm"])
        opts, over = paper_options(V, name, pr.n)
        res["paper_overrides"] = over
        ctx = V.Context.from_problem(pr, precision=prec, options=opts)
        res["paper_parameters"] = run_pbm_capped(torch, V, ctx, name, "paper", a.cap_seconds,
                                                 opts.max_outer)
        res["paper_parameters"]["precision"] = "fp64" if prec == V.VTS_FP64 else "mixed"
        ctx.close()
        if not a.paper_only:
            # this library's options target KKT <= 1e-6; its Gauss-Seidel
            # multigrid (FP32 in mixed precision) needs a positive lower bound,
            # here the one Section 7.2 uses for the interior point runs
            lib = V.default_options()
            if name.startswith("BRIDGE") and int(name.split("-")[-1]) >= 6:
                # the point-supported bridge's relative penalty floor, as for
                # the 128x64x64 bridge workload
                lib.p_min = 3e-3
            pr.rho_lo = a.library_rho_lo
            ctx = V.Context.from_problem(pr, precision=V.VTS_MIXED, options=lib)
            res["library_kkt"] = run_pbm_capped(torch, V, ctx, name, "library",
                                                a.cap_seconds, lib.max_outer)
            res["library_kkt"].update(precision="mixed", rho_lo=a.library_rho_lo, p_min=lib.p_min)
            ctx.close()
        out[name] = res
        print(f"{name}: {json.dumps(res)}", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "value": None, "unit": "see problems", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "paper problems (Section 7, Tables 3 and 4): the paper's "
                                   "parameters, then this library's (KKT <= 1e-6, mixed)",
                       "families": a.families, "levels": a.levels},
            "problems": out}
    print(json.dumps(line), flush=True)
    return 0


def scaling_run(a, torch, W, V):
    """Time-to-KKT of the benchmark cantilever family (the CANT-4-2-2-l
    geometry with the edge load of the 64x32x32 workload, V = 0.2 m) at
    refinement levels 5, 6 and 7 on one GPU, with the library's default
    options: how the solve scales with n up to 12.8 M DOFs."""
    prec = V.VTS_FP64 if a.precision == "fp64" else V.VTS_MIXED
    out = {}
    for l in a.levels:
        s2 = 2 ** (l - 1)
        pr = W.cantilever_edge(4 * s2, 2 * s2, 2 * s2, l, vol_frac=0.2)
        opts = V.default_options(eps_mr0=1e-2)
        ctx = V.Context.from_problem(pr, precision=prec, options=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status = V.VTS_OK
        for k in range(opts.max_outer):
            try:
                st = ctx.pbm_iterate()
            except V.VtsError as e:
                status = e.status
                break
            if (k + 1) % 5 == 0 or st["converged"]:
                print(f"l={l} n={pr.n}: outer {k + 1} ratio {st['ratio']:.2e} stat "
                      f"{st['stat']:.2e} t {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
            if st["converged"]:
                break
        r = ctx.pbm_solve(check=False) if status == V.VTS_OK else None
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = dict(m=pr.m, n=pr.n, seconds=dt, status=int(r["status"] if r else status),
                   device_gb=ctx.allocated_bytes() / 1e9)
        if r:
            k = device_kkt(torch, ctx, pr, ctx.state_dict()["alpha"])
            res.update(outer=r["outer"], newton=r["newton"], minres=r["minres"],
                       compliance=r["compliance"], kkt=k["kkt"],
                       ms_per_minres=dt * 1e3 / max(r["minres"], 1))
        out[f"l{l}"] = res
        print(f"l={l}: {json.dumps(res)}", file=sys.stderr, flush=True)
        ctx.close()
    line = {"metric": METRIC, "value": None, "unit": "see levels", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None,
            "dtype": "f64" if prec == V.VTS_FP64 else "f64+f32mg", "data": "synthetic",
            "config": {"workload": "cantilever 4*2^(l-1) x 2^l x 2^l, edge load, V = 0.2 m",
                       "levels": a.levels},
            "levels": out}
    print(json.dumps(line), flush=True)
    return 0


def scaling_kernels(a, torch, W, V):
    """The dominant kernels at the initial Newton point of the cantilever
    family at levels --levels, FP64 and mixed: the finest-level Gauss-Seidel
    pass, K(rho)x and the S-apply, each timed with HIP events over every
    launch of repeated calls; bandwidth from the algorithmic bytes."""
    out = {}
    for l in a.levels:
        s2 = 2 ** (l - 1)
        pr = W.cantilever_edge(4 * s2, 2 * s2, 2 * s2, l, vol_frac=0.2)
        for prec in (V.VTS_FP64, V.VTS_MIXED):
            ctx = V.Context.from_problem(pr, precision=prec)
            ctx.reset()
            ctx.newton_setup()
            g = torch.Generator(device="cpu").manual_seed(1)
            r = (torch.rand(ctx.n_dof + 1, generator=g, dtype=torch.float64) - 0.5).cuda()
            z = torch.empty_like(r)
            x = (torch.rand(ctx.n_dof, generator=g, dtype=torch.float64) - 0.5).cuda()
            y = torch.empty_like(x)
            # one untimed call of each (first use loads code and warms caches)
            ctx.precondition(r, z)
            ctx.apply_K(x, y)
            ctx.apply_S(r, z)
            torch.cuda.synchronize()
            gs = profiled(ctx, "gs_fine", lambda: [ctx.precondition(r, z) for _ in range(a.reps)])
            ka = profiled(ctx, "apply_K", lambda: [ctx.apply_K(x, y) for _ in range(a.reps)])
            sa = profiled(ctx, "apply_S", lambda: [ctx.apply_S(r, z) for _ in range(a.reps)])
            key = f"l{l}_{'fp64' if prec == V.VTS_FP64 else 'mixed'}"
            out[key] = {
                "n": pr.n, "m": pr.m,
                "gs_fine": {"avg_launch_us": gs["avg_launch_ms"] * 1e3, "gbs": gs["gbs"],
                            "frac": gs["gbs"] / HBM_PEAK_GBS,
                            "bytes_per_launch": gs["bytes_per_launch"]},
                "apply_K_f64": {"avg_launch_us": ka["avg_launch_ms"] * 1e3, "gbs": ka["gbs"],
                                "frac": ka["gbs"] / HBM_PEAK_GBS},
                "apply_S": {"avg_launch_us": sa["avg_launch_ms"] * 1e3, "gbs": sa["gbs"],
                            "frac": sa["gbs"] / HBM_PEAK_GBS},
            }
            print(f"{key}: {json.dumps(out[key])}", file=sys.stderr, flush=True)
            ctx.close()
    line = {"metric": METRIC, "value": None, "unit": "see levels", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "f64 / f64+f32mg", "data": "synthetic",
            "config": {"workload": "cantilever 4*2^(l-1) x 2^l x 2^l, initial Newton point",
                       "levels": a.levels, "reps": a.reps},
            "kernels_by_level": out}
    print(json.dumps(line), flush=True)
    return 0


def _timed(torch, fn, reps):
    """Average milliseconds of fn() over reps calls, HIP events on the
    current stream (the library's default stream)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline_one_case_K(pr):
    """The FP64 oracle's K(rho)u (element gather, dense element products,
    scatter) applied once to one load case of `pr` on the host cores."""
    import workloads as W
    from oracle import fe
    gr = fe.Grid(pr.nx, pr.ny, pr.nz, pr.fixed)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    rh = W.random_rho(pr.m, seed=1)
    xv = W.random_vector(pr.n_dof, seed=2)
    t = time.perf_counter()
    fe.apply_K(gr, Ke, rh, xv)
    cpu_s = time.perf_counter() - t
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return {"value": pr.n_dof / cpu_s / 1e9, "unit": "GDOF/s (K(rho)u)", "cores": cores,
            "kind": "oracle",
            "sample": f"one application of the oracle's K(rho)u to one case of {pr.name} "
                      f"({cpu_s:.2f} s)"}


def multiload_ttk(torch, W, V, pr2):
    """Time-to-KKT (FP64) of a multi-load problem from the initial point (the
    second of two solves), and the KKT residual of the returned state on the
    device: equilibrium of every case, volume, stationarity with the summed
    energies."""
    import numpy as np
    c2 = V.Context.from_problem(pr2, precision=V.VTS_FP64,
                                options=V.default_options(eps_mr0=1e-2))
    c2.pbm_solve()
    c2.reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = c2.pbm_solve()
    torch.cuda.synchronize()
    ttk = time.perf_counter() - t
    d = c2.state_dict()
    cases = W.load_cases(pr2)
    F = np.where(np.tile(pr2.fixed, len(cases)) == 1, 0.0, cases.ravel())
    u = torch.as_tensor(d["u"], device="cuda")
    y = torch.empty_like(u)
    c2.apply_K(u, y)
    e = torch.empty(pr2.m, dtype=torch.float64, device="cuda")
    c2.element_energy(u, e)
    torch.cuda.synchronize()
    Ft = torch.as_tensor(F, device="cuda")
    rho = torch.as_tensor(d["rho"], device="cuda")
    lam = d["alpha"]
    proj = torch.clamp(rho + (e - lam) / lam, pr2.rho_lo, pr2.rho_hi)
    r_box = float(torch.clamp(torch.maximum(pr2.rho_lo - rho, rho - pr2.rho_hi), min=0.0).max())
    kkt = max(float(torch.linalg.norm(y - Ft) / torch.linalg.norm(Ft)),
              float(abs(rho.sum() - pr2.V) / pr2.V), r_box / pr2.rho_hi,
              float(((rho - proj).abs() / pr2.rho_hi).max()))
    c2.close()
    print(f"time-to-KKT {pr2.name}: {ttk:.2f} s, outer {res['outer']} newton {res['newton']} "
          f"minres {res['minres']} KKT {kkt:.2e}", file=sys.stderr, flush=True)
    return {"workload": pr2.name, "seconds": ttk, "outer": res["outer"],
            "newton": res["newton"], "minres": res["minres"], "kkt": kkt,
            "status": res["status"], "compliance": res["compliance"]}


def multiload_run(a, torch, W, V):
    """Several load cases (the stacked problem, summed compliance), FP64.
    (1) The three point loads of the 192x96x96 cantilever as three cases, at
    the initial Newton point: MINRES-MG iterations per second on the stacked
    system (the line's value), the finest colour pass of its V-cycle (node
    blocks of 9 unknowns; HIP events around every launch, algorithmic bytes)
    as the roofline kernel, the multigrid setup, the stacked S-apply, one
    V-cycle, and K(rho) on the three cases (one element-kernel launch per
    case) over rotating (x, rho, y) sets.  (2) Time-to-KKT of the two-case
    64x32x32 cantilever, KKT from the returned state on the device.  (3) The
    CPU oracle's K(rho)u on one case of workload (1)."""
    import numpy as np
    pr = W.multi_config(2)
    its = 40
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64,
                                 options=V.default_options(max_minres=its))
    k, nvec, m, nd = ctx.nload, ctx.n_vec, ctx.m, ctx.n_dof
    g = torch.Generator(device="cpu").manual_seed(1)
    sets = 4
    xs = [(torch.rand(nvec, generator=g, dtype=torch.float64) - 0.5).cuda() for _ in range(sets)]
    ys = [torch.empty_like(xs[0]) for _ in range(sets)]
    rhos = [(0.001 + 0.999 * torch.rand(m, generator=g, dtype=torch.float64)).cuda()
            for _ in range(sets)]
    reps = max(a.reps, 1)
    state = {"q": 0}

    def batched():
        q = state["q"] = (state["q"] + 1) % sets
        ctx.apply_K_rho(rhos[q], xs[q], ys[q])

    k_ms = _timed(torch, batched, reps * sets)
    k_launch_bytes = 16.0 * nd + 8.0 * m
    k_gbs = k * k_launch_bytes / (k_ms * 1e-3) / 1e9
    k_gdofs = nvec / (k_ms * 1e-3) / 1e9
    print(f"K(rho) on {k} cases: {k_ms * 1e3:.1f} us per call ({k} launches), {k_gdofs:.1f} "
          f"GDOF/s, {k_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    for q in range(sets):
        xs[q] = ys[q] = rhos[q] = None
    torch.cuda.empty_cache()
    # the stacked Newton system at the initial point
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.newton_setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    r = (torch.rand(nvec + 1, generator=g, dtype=torch.float64) - 0.5).cuda()
    z = torch.empty_like(r)
    sa_ms = _timed(torch, lambda: ctx.apply_S(r, z), reps)
    vc_ms = _timed(torch, lambda: ctx.precondition(r, z), reps)
    gs = profiled(ctx, "gs_fine", lambda: [ctx.precondition(r, z) for _ in range(reps)])
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = ctx.solve_newton(0.0)
    torch.cuda.synchronize()
    mr_s = time.perf_counter() - t
    mr_rate = st["iterations"] / mr_s
    print(f"setup {setup_s:.2f} s, S-apply {sa_ms * 1e3:.0f} us, V-cycle {vc_ms:.2f} ms, finest "
          f"colour pass {gs['avg_launch_ms'] * 1e3:.1f} us ({gs['gbs']:.0f} GB/s), MINRES-MG "
          f"{mr_rate:.1f} it/s", file=sys.stderr, flush=True)
    ctx.close()
    torch.cuda.empty_cache()

    # (2) time-to-KKT of the two-case cantilever
    pr2 = W.multi_config(1)
    ttk_out = None
    if not a.ml_no_solve:
        ttk_out = multiload_ttk(torch, W, V, pr2)

    # (3) the oracle's K(rho)u on one case of workload (1)
    cpu = cpu_baseline_one_case_K(pr)

    # plain copies of 256 MiB: the scale reference of the traffic counters
    buf = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(buf)
    for _ in range(5):
        dst.copy_(buf)
    torch.cuda.synchronize()
    del buf, dst

    kern = f"k_ml_gs<{3 * k}, true>"
    line = {
        "metric": "MINRES-MG iterations/s on the stacked Newton system of k load cases",
        "value": mr_rate, "unit": "iterations/s (FP64, 3 load cases, 192x96x96)",
        "n_gpus": 1, "steps": st["iterations"], "warmup": 1, "ms_per_step": 1e3 * mr_s / max(st["iterations"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{pr.name} (the three point loads as three load cases)",
                   "load_cases": k, "n_dof_per_case": nd, "m": m},
        "roofline": {"bound": "hbm", "achieved": gs["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gs["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(pr.name, kern),
                     "kernel": kern, "algorithmic_bytes_per_launch": gs["bytes_per_launch"],
                     "avg_launch_us": gs["avg_launch_ms"] * 1e3, "launches": gs["launches"]},
        "cpu_baseline": cpu,
        "multiload": {
            "K_3_cases_us": k_ms * 1e3, "K_gdofs": k_gdofs,
            "K_roofline": {"kernel": "k_apply_K_plane<double>", "achieved": k_gbs,
                           "frac": k_gbs / HBM_PEAK_GBS,
                           "traffic": measured_traffic("cant3pt-192x96x96",
                                                       "k_apply_K_plane<double>")},
            "setup_s_initial_point": setup_s, "apply_S_us": sa_ms * 1e3,
            "vcycle_ms": vc_ms, "minres_mg_iters_per_s": mr_rate,
            "time_to_kkt": ttk_out,
        },
    }
    print(json.dumps(line), flush=True)
    return 0


def device_kkt(torch, ctx, pr, lam):
    """KKT residual of the context's (rho, u) with volume multiplier lam, by
    its definition: r_eq = ||K(rho)u - f||/||f||, r_vol = |sum rho - V|/V,
    r_box, and r_stat = max_i |rho_i - clip(rho_i + (e_i - lam)/lam)|/hi_i,
    with K(rho)u and e_i from vts_apply_K and vts_element_energy."""
    dev = "cuda"
    u = ctx.vector("u")
    rho = ctx.vector("rho")
    fixed = torch.as_tensor(np.asarray(pr.fixed, dtype=bool), device=dev)
    f = torch.as_tensor(np.asarray(pr.f, dtype=np.float64), device=dev).masked_fill(fixed, 0.0)
    m = rho.numel()
    lo = torch.as_tensor(np.broadcast_to(np.asarray(pr.rho_lo, float), (m,)).copy(), device=dev)
    hi = torch.as_tensor(np.broadcast_to(np.asarray(pr.rho_hi, float), (m,)).copy(), device=dev)
    y = torch.empty_like(u)
    ctx.apply_K(u, y)
    e = torch.empty_like(rho)
    ctx.element_energy(u, e)
    torch.cuda.synchronize()
    r_eq = float(torch.linalg.norm(y - f) / torch.linalg.norm(f))
    r_vol = float(abs(rho.sum() - pr.V) / pr.V)
    r_box = float(torch.clamp(torch.maximum(lo - rho, rho - hi), min=0.0).max() / hi.max())
    proj = torch.minimum(torch.maximum(rho + (e - lam) / lam, lo), hi)
    r_stat = float(((rho - proj).abs() / hi).max())
    return dict(r_eq=r_eq, r_vol=r_vol, r_box=r_box, r_stat=r_stat,
                kkt=max(r_eq, r_vol, r_box, r_stat))


def ip_compare(a, torch, W, V):
    """The primal-dual interior point method (Algorithm 3, the paper's
    parameters: eps_IP 1e-5, sigma 0.2, r = s = 1e-2 initially) and PBM on
    the same workload, both on the GPU in FP64."""
    pr = W.config(a.workload)
    eps_mr0 = pr.extra.get("eps_mr0")
    opts = V.default_options()
    if eps_mr0:
        opts.eps_mr0 = eps_mr0
    if pr.extra.get("p_min"):
        opts.p_min = pr.extra["p_min"]
    ctx = V.Context.from_problem(pr, precision=V.VTS_FP64, options=opts)
    ctx.reset()
    ctx.pbm_solve()
    torch.cuda.synchronize()
    ctx.reset()
    t0 = time.perf_counter()
    r = ctx.pbm_solve()
    torch.cuda.synchronize()
    t_pbm = time.perf_counter() - t0
    k_pbm = device_kkt(torch, ctx, pr, ctx.state_dict()["alpha"])
    print(f"PBM: {t_pbm:.2f} s, {r['outer']} outer, {r['newton']} Newton, {r['minres']} MINRES",
          file=sys.stderr, flush=True)
    # IP iterations one call at a time, so that progress is visible
    t0 = time.perf_counter()
    ctx.ip_init()
    its, mr, status, hist = 0, 0, V.VTS_ENOTCONV, []
    s = {}
    for k in range(300):
        s = ctx.ip_step(check=False)
        its, mr = k + 1, mr + s["minres_its"]
        hist.append(s["minres_its"])
        print(f"IP iteration {its}: minres {s['minres_its']} gap ratio {s['gap_ratio']:.2e} "
              f"res_IP {s['res_ip']:.2e} eps_MR {s['eps_mr']:.1e}", file=sys.stderr, flush=True)
        if s["status"] != V.VTS_OK:
            status = s["status"]
            break
        if s["converged"]:
            status = V.VTS_OK
            break
    torch.cuda.synchronize()
    t_ip = time.perf_counter() - t0
    k_ip = device_kkt(torch, ctx, pr, -ctx.state_dict()["alpha"])
    line = {
        "metric": METRIC, "value": 1.0 / t_ip, "unit": "IP solves/s (eps_IP 1e-5)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": t_ip * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": pr.name, "method": "primal-dual IP (Algorithm 3)",
                   "eps_ip": 1e-5, "sigma": 0.2, "max_minres": 3000},
        "ip": {"seconds": t_ip, "iterations": its, "minres": mr, "status": status,
               "compliance": s.get("compliance"), "gap_ratio": s.get("gap_ratio"),
               "res_ip": s.get("res_ip"), "kkt": k_ip["kkt"], "kkt_terms": k_ip,
               "minres_per_iteration": hist},
        "pbm": {"seconds": t_pbm, "outer": r["outer"], "newton": r["newton"],
                "minres": r["minres"], "compliance": r["compliance"], "kkt": k_pbm["kkt"]},
        "ip_over_pbm_time": t_ip / t_pbm,
        "ip_compliance_excess": ((s["compliance"] - r["compliance"]) / r["compliance"]
                                 if s.get("compliance") else None),
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def doc_compare(a, torch, W, V):
    """DOC (Algorithm 4, q = 0.5, eps_DOC = 1e-3, bisection tolerance
    1e-4) and PBM on the same workload, both on the GPU."""
    pr = W.config(a.workload)
    prec = V.VTS_MIXED if pr.extra.get("precision") == "mixed" else V.VTS_FP64
    eps_mr0 = pr.extra.get("eps_mr0")
    opts = V.default_options()
    if eps_mr0:
        opts.eps_mr0 = eps_mr0
    ctx = V.Context.from_problem(pr, precision=prec, options=opts)
    ctx.reset()
    ctx.pbm_solve()
    torch.cuda.synchronize()
    ctx.reset()
    t0 = time.perf_counter()
    r = ctx.pbm_solve()
    torch.cuda.synchronize()
    t_pbm = time.perf_counter() - t0
    print(f"PBM: {t_pbm:.2f} s, {r['outer']} outer, {r['newton']} Newton", file=sys.stderr,
          flush=True)
    # DOC iterations one call at a time, so that progress is visible
    ctx.reset()
    t0 = time.perf_counter()
    d = dict(iterations=0, minres_its=0, status=V.VTS_ENOTCONV)
    for k in range(5000):
        s = ctx.doc_step(q=0.5, tau=1e-4, eps_doc=1e-3, eps_mr=1e-6)
        d["iterations"] = k + 1
        d["minres_its"] += s["minres_its"]
        if (k + 1) % 20 == 0:
            print(f"DOC iteration {k + 1}: change {s['change']:.2e} compliance "
                  f"{s['compliance']:.6f} minres {s['minres_its']}", file=sys.stderr, flush=True)
        if s["converged"]:
            d["status"] = V.VTS_OK
            break
    torch.cuda.synchronize()
    t_doc = time.perf_counter() - t0
    # 1/2 f^T u of the last iteration: at convergence rho is kept, so this is
    # the compliance of the returned design (to the MINRES tolerance)
    c_doc = s["compliance"]
    line = {
        "metric": METRIC, "value": 1.0 / t_doc, "unit": "DOC solves/s (eps_DOC 1e-3)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": t_doc * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == V.VTS_FP64 else "f64+f32mg", "data": "synthetic",
        "config": {"workload": pr.name, "method": "DOC (Algorithm 4)", "q": 0.5,
                   "eps_doc": 1e-3, "eps_mr": 1e-6},
        "doc": {"seconds": t_doc, "iterations": d["iterations"], "minres": d["minres_its"],
                "status": d["status"], "compliance": c_doc},
        "pbm": {"seconds": t_pbm, "outer": r["outer"], "newton": r["newton"],
                "minres": r["minres"], "compliance": r["compliance"]},
        "doc_over_pbm_time": t_doc / t_pbm,
        "doc_compliance_excess": (c_doc - r["compliance"]) / r["compliance"],
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def serving(a, torch, W, V):
    """Latency of a Poisson stream of mixed requests (grids 16x8x8 .. 96x48x48,
    cantilever edge / bridge face loads, V/m ~ U[0.1, 0.4]) at three arrival
    rates, relative to the mean service time of the mix run alone."""
    from paper_1904_06556_amd import serve
    # serving policy: the library's options with a 500-iteration outer budget;
    # the point-supported bridges take the relative penalty floor 5e-3 |alpha|
    cant_opts = V.default_options(max_outer=500)
    bridge_opts = V.default_options(p_min=5e-3, max_outer=500)

    def opts(pr):
        return bridge_opts if pr.name.startswith("bridge") else cant_opts
    if a.burst is not None:
        return serving_burst(a, torch, W, V, opts)
    base = W.serving_requests(a.requests, rate=1.0, seed=0)
    probs = [p for _, p in base]
    n_alone = min(8, len(probs))
    alone = serve.time_alone(probs[:n_alone], precision=V.VTS_MIXED, options=opts)
    for r, p in zip(alone, probs):
        print(f"alone {p.name} status {r['status']} service {r['service']:.2f} s",
              file=sys.stderr, flush=True)
    t_alone = a.t_alone if a.t_alone else float(np.mean([r["service"] for r in alone]))
    pool = int(a.pool_gb * (1 << 30))
    rates = {}
    same = True
    for factor in a.rates:
        lam = factor / t_alone
        reqs = W.serving_requests(a.requests, rate=lam, seed=0)
        srv = V.Server(a.slots, pool, batching=not a.no_batching)
        recs = serve.run_stream(srv, reqs, precision=V.VTS_MIXED, options=opts,
                                on_done=lambda r: print(
                                    f"  rate x{factor}: request {r['index']} status {r['status']} "
                                    f"latency {r['latency']:.2f} s", file=sys.stderr, flush=True))
        gstats = srv.group_stats()
        srv.close()
        for k in range(n_alone):
            same &= (recs[k]["compliance"] == alone[k]["compliance"] and
                     recs[k]["minres"] == alone[k]["minres"])
        rates[f"x{factor}"] = dict(rate_per_s=lam, **serve.summarize(recs),
                                   batching=gstats if not a.no_batching else None)
    mid = rates.get("x0.8") or rates[f"x{a.rates[0]}"]
    line = {
        "metric": METRIC, "value": mid["throughput_per_s"],
        "unit": "VTS solves/s (served stream at 0.8 x capacity of one-at-a-time service)",
        "n_gpus": 1, "steps": a.requests, "warmup": 0,
        "ms_per_step": 1e3 / mid["throughput_per_s"] if mid["throughput_per_s"] else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32mg", "data": "synthetic",
        "config": {"workload": "serving stream", "grids": [list(g) for g in W.SERVING_GRIDS],
                   "requests_per_rate": a.requests, "slots": a.slots, "pool_gb": a.pool_gb,
                   "precision": "mixed", "p_min_cantilever": cant_opts.p_min,
                   "p_min_bridge": bridge_opts.p_min, "max_outer": cant_opts.max_outer,
                   "batching": not a.no_batching, "rates": a.rates},
        "p50_s": mid["p50_s"], "p99_s": mid["p99_s"],
        "mean_service_alone_s": t_alone, "rates": rates,
        "mix_equals_alone": bool(same),
    }
    print(json.dumps(line), flush=True)
    return 0


def burst_problems(W, grid, n):
    """n requests of serving grid `grid` (loads alternating, V/m ~ U[0.1, 0.4], seed 1)."""
    nx, ny, nz, l = W.SERVING_GRIDS[grid]
    rng = np.random.default_rng(1)
    probs = []
    for k in range(n):
        frac = float(rng.uniform(0.1, 0.4))
        probs.append(W.cantilever_edge(nx, ny, nz, l, vol_frac=frac) if k % 2 == 0 else
                     W.bridge_top(nx, ny, nz, l, vol_frac=frac, h=2.0 ** (1 - l)))
    return probs


def burst_once(V, serve, probs, slots, pool, batching, opts):
    """All of probs submitted at once to a server; latency percentiles,
    throughput and the group runners' counters."""
    srv = V.Server(slots, pool, batching=batching)
    t0 = time.perf_counter()
    recs = serve.run_stream(srv, [(0.0, p) for p in probs], precision=V.VTS_MIXED,
                            options=opts, keep_fields=True)
    wall = time.perf_counter() - t0
    g = srv.group_stats()
    srv.close()
    lat = np.array([r["latency"] for r in recs])
    return recs, dict(wall_s=wall, solves_per_s=len(recs) / wall,
                      ok=int(sum(r["status"] == V.VTS_OK for r in recs)),
                      p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                      group_stats=g if batching else None)


def serving_burst(a, torch, W, V, opts):
    """--burst G: a.requests requests of serving grid G (cantilever edge and
    bridge face loads, V/m ~ U[0.1, 0.4]) all submitted at once, served by
    a.slots workers with batching on and then off: time until the last
    result, and the group runners' mean batch."""
    from paper_1904_06556_amd import serve
    nx, ny, nz, l = W.SERVING_GRIDS[a.burst]
    probs = burst_problems(W, a.burst, a.requests)
    pool = int(a.pool_gb * (1 << 30))
    out, results = {}, {}
    for batching in (True, False):
        key = "batching" if batching else "no_batching"
        results[key], out[key] = burst_once(V, serve, probs, a.slots, pool, batching, opts)
        print(f"burst {key}: {json.dumps(out[key])}", file=sys.stderr, flush=True)
    same = all(x["compliance"] == y["compliance"] and np.array_equal(x["rho"], y["rho"])
               for x, y in zip(results["batching"], results["no_batching"]))
    line = {"metric": METRIC, "value": out["batching"]["solves_per_s"],
            "unit": "VTS solves/s (burst of same-grid requests, batching on)",
            "n_gpus": 1, "steps": a.requests, "warmup": 0,
            "ms_per_step": 1e3 * out["batching"]["wall_s"] / a.requests,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64+f32mg", "data": "synthetic",
            "config": {"workload": f"burst of {a.requests} requests on {nx}x{ny}x{nz} l{l}",
                       "slots": a.slots, "precision": "mixed"},
            "burst": out, "batched_equals_unbatched": bool(same),
            "speedup": out["no_batching"]["wall_s"] / out["batching"]["wall_s"]}
    print(json.dumps(line), flush=True)
    return 0


def solve_run(a, torch, W, V):
    """Time-to-KKT of complete PBM solves of --workload (the initial point
    re-set on the device before each solve)."""
    pr = W.config(a.workload)
    eps_mr0 = pr.extra.get("eps_mr0")
    opts = V.default_options()
    if eps_mr0:
        opts.eps_mr0 = eps_mr0
    if pr.extra.get("p_min"):
        opts.p_min = pr.extra["p_min"]
    want = pr.extra.get("precision") if a.precision == "config" else a.precision
    prec = V.VTS_MIXED if want == "mixed" else V.VTS_FP64
    ctx = V.Context.from_problem(pr, precision=prec, options=opts)
    torch.cuda.synchronize()

    for w in range(a.warmup):
        ctx.reset()
        r = ctx.pbm_solve()
        print(f"warmup {w}: outer {r['outer']} newton {r['newton']} minres {r['minres']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ctx.reset()
        results.append(ctx.pbm_solve())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"timed: {a.steps} solves in {t1 - t0:.2f} s", file=sys.stderr, flush=True)
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    last = results[-1]

    # KKT of the last result by its definition, from the library's own
    # operators on the device
    k = device_kkt(torch, ctx, pr, ctx.state_dict()["alpha"])
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_{pr.name}.json")
    c_err = None
    if os.path.exists(gold):
        g = json.load(open(gold))
        c_err = abs(last["compliance"] - g["compliance_half_fu"]) / g["compliance_half_fu"]

    # dominant kernel (Gauss-Seidel colour pass on the finest level) and the
    # S-apply, each timed over every launch of one further complete solve
    def solve_again():
        ctx.reset()
        ctx.pbm_solve()
    gs = profiled(ctx, "gs_fine", solve_again)
    sa = profiled(ctx, "apply_S", solve_again)
    print(f"profiled: gs_fine {gs['launches']} launches {gs['avg_launch_ms'] * 1e3:.2f} us, "
          f"apply_S {sa['launches']} launches {sa['avg_launch_ms'] * 1e3:.2f} us",
          file=sys.stderr, flush=True)
    mr_rate, mr_its = minres_rate(torch, ctx)
    bytes_per, kr = kernel_roofline(torch, ctx, pr)
    rot = kr["rotating"]
    gs_kernel = "k_gs_mf<double>" if prec == V.VTS_FP64 else "k_gs_mf<float>"
    line = {
        "metric": METRIC,
        "value": 1e3 / ms_per_step,
        "unit": "VTS solves/s (1/time-to-KKT)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == V.VTS_FP64 else "f64+f32mg",
        "data": "synthetic",
        "config": {"workload": pr.name, "grid": [pr.nx, pr.ny, pr.nz], "levels": pr.levels,
                   "m": pr.m, "n": pr.n, "V_over_m": pr.V / pr.m,
                   "precision": "fp64" if prec == V.VTS_FP64 else "mixed",
                   "eps_mr0": eps_mr0, "parallelism": "1 GPU"},
        "time_to_kkt_s": ms_per_step / 1e3,
        "kkt": k["kkt"], "kkt_terms": k,
        "compliance": last["compliance"], "compliance_rel_err_vs_oracle": c_err,
        "outer": last["outer"], "newton": last["newton"], "minres": last["minres"],
        "k_apply_gdofs": rot["gdofs"], "k_apply_gdofs_hot_cache": kr["hot"]["gdofs"],
        "minres_mg_iters_per_s": mr_rate,
        "roofline": {"kernel": f"{gs_kernel} (finest-level multicolour block "
                               "Gauss-Seidel pass, matrix-free)",
                     "bound": "hbm", "achieved": gs["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gs["gbs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(pr.name, gs_kernel),
                     "bytes_per_launch": gs["bytes_per_launch"],
                     "avg_launch_ms": gs["avg_launch_ms"], "launches": gs["launches"]},
        "kernels": {
            "apply_S_tile": {"avg_launch_ms": sa["avg_launch_ms"], "gbs": sa["gbs"],
                             "bytes_per_launch": sa["bytes_per_launch"],
                             "launches_per_solve": sa["launches"]},
            "apply_K_tile_f64": {"avg_launch_ms": rot["ms"], "gbs": rot["gbs"],
                                 "gdofs": rot["gdofs"], "bytes_per_launch": bytes_per,
                                 "buffers": "rotating, working set > 512 MB"},
            "gs_fine_launches_per_solve": gs["launches"]},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pr, eps_mr0, last["newton"], a.cpu_seconds)
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


HEADLINE_WORKLOAD = 3      # cantilever 192x96x96, three point loads, mixed precision
K_SET_BYTES = 1.0e9        # rotating K(rho)u sets: more than the 256 MB Infinity Cache
def cpu_baseline_k_apply(pr, budget_s):
    """The FP64 oracle's K(rho)u (element gather, dense 24x24 element
    products, scatter by bincount) on the same grid, repeated for about
    budget_s seconds on the host cores."""
    from oracle import fe
    g = fe.Grid(pr.nx, pr.ny, pr.nz, pr.fixed)
    Ke = fe.element_stiffness(pr.E, pr.nu, pr.h)
    import workloads as W
    rho = W.random_rho(pr.m, seed=1)
    x = W.random_vector(pr.n_dof, seed=2)
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((d.get("num_threads") or 1) for d in threadpool_info()) or None
    except Exception:
        pass
    t0 = time.perf_counter()
    n = 0
    while True:
        fe.apply_K(g, Ke, rho, x)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / n
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count()
    return dict(value=pr.n_dof / dt / 1e9, unit="GDOF/s (K(rho)u, FP64)",
                cores=threads or 1, cores_available=avail, kind="oracle",
                seconds_per_apply=dt, applications=n,
                sample=(f"{n} applications of the oracle's K(rho)u (gather, 24x24 element "
                        f"products through BLAS with {threads or 1} threads, bincount "
                        f"scatter on one thread) on the same {pr.name} grid, random x and "
                        f"rho"))


def headline(a, torch, W, V):
    """Default run: the 192x96x96 three-load cantilever.  A step is one outer
    PBM iteration (mixed precision) plus K(rho)u on the rotating FP64 sets."""
    pr = W.config(HEADLINE_WORKLOAD)
    stream = torch.cuda.Stream()
    opts = V.default_options()
    ctx = V.Context.from_problem(pr, precision=V.VTS_MIXED, options=opts, stream=stream)
    ctxk = V.Context.from_problem(pr, precision=V.VTS_FP64, options=opts, stream=stream)
    nd, m = ctx.n_dof, ctx.m
    k_bytes = 16.0 * nd + 8.0 * m          # read x and rho, write y (8 B each)
    nsets = max(8, int(math.ceil(K_SET_BYTES / k_bytes)))
    gen = torch.Generator(device="cpu").manual_seed(1)
    xs, rhos, ys = [], [], []
    for _ in range(nsets):
        xs.append((2.0 * torch.rand(nd, generator=gen, dtype=torch.float64) - 1.0).cuda())
        rhos.append((1e-3 + (1.0 - 1e-3) * torch.rand(m, generator=gen,
                                                        dtype=torch.float64)).cuda())
        ys.append(torch.empty(nd, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()

    # K(rho)u is timed by HIP events recorded on the stream both contexts
    # launch on, around each step's back-to-back launches
    k_events = []

    def k_batch():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(nsets):
            ctxk.apply_K_rho(rhos[i], xs[i], ys[i])
        e1.record(stream)
        k_events.append((e0, e1))

    def step():
        st = ctx.pbm_iterate()
        k_batch()
        return st

    for w in range(a.warmup):
        st = step()
        print(f"warmup {w}: outer iteration newton {st['newton_its']} minres "
              f"{st['minres_its']} ratio {st['ratio']:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    k_events.clear()
    stats = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        stats.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kp = {"launches": nsets * len(k_events),
          "total_ms": sum(e0.elapsed_time(e1) for e0, e1 in k_events)}
    wall = t1 - t0
    k_ms = kp["total_ms"] / max(kp["launches"], 1)
    k_gdofs = nd / (k_ms * 1e-3) / 1e9
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9
    minres = sum(s["minres_its"] for s in stats)
    newton = sum(s["newton_its"] for s in stats)
    print(f"timed: {a.steps} steps in {wall:.2f} s; K(rho)u {kp['launches']} launches "
          f"{k_ms * 1e3:.2f} us; {newton} Newton steps, {minres} MINRES iterations",
          file=sys.stderr, flush=True)

    # the other kernels of the hot path over one more outer iteration
    def one_iteration():
        ctx.pbm_iterate()
    gs = profiled(ctx, "gs_fine", one_iteration)
    sa = profiled(ctx, "apply_S", one_iteration)

    # MINRES-MG at a fixed Newton point (the current state), fixed count
    def fixed_point_rate(c):
        c.newton_setup()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = c.solve_newton(0.0)
        torch.cuda.synchronize()
        return r["iterations"] / (time.perf_counter() - t), r["iterations"]
    mr_mixed, mr_its = fixed_point_rate(ctx)
    ctxk.set_state(ctx.get_state())
    mr_fp64, _ = fixed_point_rate(ctxk)
    print(f"fixed-point MINRES-MG: mixed {mr_mixed:.1f} it/s, FP64 {mr_fp64:.1f} it/s",
          file=sys.stderr, flush=True)
    ctx.close()
    ctxk.close()
    del xs, rhos, ys

    # time-to-KKT of the 64x32x32 cantilever, FP64 and mixed
    pr2 = W.config(1)
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_{pr2.name}.json")
    c_or = json.load(open(gold))["compliance_half_fu"] if os.path.exists(gold) else None
    ttk = {}
    for name, prec in (("fp64", V.VTS_FP64), ("mixed", V.VTS_MIXED)):
        o2 = V.default_options(eps_mr0=pr2.extra["eps_mr0"])
        tc = time.perf_counter()
        c2 = V.Context.from_problem(pr2, precision=prec, options=o2)
        r = c2.pbm_solve()
        torch.cuda.synchronize()
        t_create = time.perf_counter() - tc
        runs = []
        for _ in range(2):
            c2.reset()
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = c2.pbm_solve()
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t)
        k = device_kkt(torch, c2, pr2, c2.state_dict()["alpha"])
        ttk[name] = dict(seconds=min(runs), seconds_from_create=t_create,
                         outer=r["outer"], newton=r["newton"], minres=r["minres"],
                         kkt=k["kkt"], compliance=r["compliance"],
                         compliance_rel_err_vs_oracle=(abs(r["compliance"] - c_or) / c_or
                                                       if c_or else None))
        print(f"time-to-KKT {pr2.name} {name}: {min(runs):.3f} s (from vts_create "
              f"{t_create:.3f} s) KKT {k['kkt']:.2e}", file=sys.stderr, flush=True)
        c2.close()

    line = {
        "metric": METRIC,
        "value": k_gdofs,
        "unit": "GDOF/s (K(rho)u, FP64, rotating sets beyond the Infinity Cache)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": pr.name, "grid": [pr.nx, pr.ny, pr.nz], "levels": pr.levels,
                   "m": pr.m, "n": pr.n, "n_dof": nd, "V_over_m": pr.V / pr.m,
                   "hot_path_precision": "mixed (FP32 multigrid, FP64 MINRES/Newton/PBM)",
                   "k_sets": nsets, "k_set_bytes": nsets * (k_bytes + 8.0 * nd),
                   "step": "one outer PBM iteration + K(rho)u on every set",
                   "parallelism": "1 GPU"},
        "roofline": {"kernel": "k_apply_K_plane<double> (K(rho)x, FP64)",
                     "bound": "hbm", "achieved": k_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": k_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(pr.name, "k_apply_K_plane<double>"),
                     "bytes_per_launch": k_bytes, "avg_launch_ms": k_ms,
                     "launches": kp["launches"]},
        "hot_path": {"outer_iterations_per_s": a.steps / wall,
                     "minres_mg_iters_per_s": minres / wall,
                     "newton_steps": newton, "minres_iterations": minres,
                     "last_gap_ratio": stats[-1]["ratio"], "last_stat": stats[-1]["stat"],
                     "minres_mg_fixed_point_iters_per_s": {"mixed": mr_mixed, "fp64": mr_fp64,
                                                           "iterations": mr_its}},
        "kernels": {
            "gs_fine": {"kernel": "k_gs_mf<float>",
                        "avg_launch_ms": gs["avg_launch_ms"], "gbs": gs["gbs"],
                        "bytes_per_launch": gs["bytes_per_launch"],
                        "traffic": measured_traffic(pr.name, "k_gs_mf<float>"),
                        "launches_per_outer_iteration": gs["launches"],
                        "precision": "fp32"},
            "apply_S": {"kernel": "k_S_plane<double, 0>",
                        "avg_launch_ms": sa["avg_launch_ms"], "gbs": sa["gbs"],
                        "bytes_per_launch": sa["bytes_per_launch"],
                        "traffic": measured_traffic(pr.name, "k_S_plane<double, 0>"),
                        "launches_per_outer_iteration": sa["launches"]}},
        "time_to_kkt_cant-64x32x32": ttk,
        "mixed_over_fp64_time_to_kkt": ttk["mixed"]["seconds"] / ttk["fp64"]["seconds"],
    }
    # serving latency: a burst of 32 requests of the 16x8x8 serving grid
    # through the request loop, 16 slots, batching on
    from paper_1904_06556_amd import serve
    sopts = V.default_options(max_outer=500)
    _, sb = burst_once(V, serve, burst_problems(W, 0, 32), 16, 4 << 30, True,
                       lambda p: V.default_options(p_min=5e-3, max_outer=500)
                       if p.name.startswith("bridge") else sopts)
    line["serving_burst_32x16x8x8"] = sb
    print(f"serving burst: {json.dumps(sb)}", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_k_apply(pr, a.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {a.gpus} is not supported "
              f"(the path runs on one GPU; there is no multi-GPU code)", file=sys.stderr)
        return 2
    import torch
    import workloads as W
    from paper_1904_06556_amd import vts as V

    if a.kernels:
        return kernels_only(a, torch, W, V)
    if a.serve:
        return serving(a, torch, W, V)
    if a.doc:
        return doc_compare(a, torch, W, V)
    if a.scale_kernels:
        return scaling_kernels(a, torch, W, V)
    if a.multiload:
        return multiload_run(a, torch, W, V)
    if a.scale:
        return scaling_run(a, torch, W, V)
    if a.paper and a.ip:
        return paper_problems_ip(a, torch, W, V)
    if a.ip:
        return ip_compare(a, torch, W, V)
    if a.paper:
        return paper_problems(a, torch, W, V)
    if a.solve:
        return solve_run(a, torch, W, V)
    return headline(a, torch, W, V)


if __name__ == "__main__":
    sys.exit(main())
