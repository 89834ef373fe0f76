#!/usr/bin/env python3
"""Throughput of the generalized Poisson / Poisson-Boltzmann solver on one MI355X.

Workload (default, `--workload charged_solute`): nonlinear Poisson-Boltzmann
for a charged solute, free boundaries, 160^3 grid, h = 0.3 bohr (FFT lengths
320), 48 Gaussian charges (sigma in U[0.6, 1.2], q in U[-1, 1] shifted to a
net +4, centres in a 6-bohr ball, seed 4) in a density-dependent (sccs)
cavity, 1 M 1:1 electrolyte with steric ions (p = 0.74, R = 3 A) excluded
where eps < eps0, Algorithm SCPBimproved with mixing 0.15, outer tolerance
1e-6, inner PCG iterations to the absolute residual the algorithm sets;
mixed precision (FP32 FFT passes and vectors, FP64 inner products and
solution).

One step = one complete solve on inputs already resident in HBM: the
per-request fields (sqrt(eps), q), every outer step with its inner PCG
iterations and ionic update, and the energy.  The plan (Green's spectrum,
buffers, captured graphs) is built before the timed region.

Prints ONE JSON line: solves/s as `value`, Mgridpts*iter/s over all inner
iterations, p50/p99 latency, the FP64 one-at-a-time comparator, the roofline
of the dominant pass (timed live with HIP events on the solve stream), the
oracle's accuracy check at 1e-10 and its timing on the host cores, plus the
molecule 96^3 line and the serving stream's latencies as extra keys.
Other workloads: molecule (96^3 generalized Poisson), slab (128x128x192
surface, linear PB), serving, rigid, sc.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

PASSES = ("xfwd", "yfwd", "zconv", "yinv", "xinv")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed solves (default: 10 for charged_solute, 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="charged_solute",
                    choices=("charged_solute", "molecule", "slab", "serving", "rigid", "sc",
                             "micro", "refine"),
                    help="charged_solute: nonlinear PB at 160^3 (default); molecule: "
                         "generalized Poisson at 96^3; slab: linear PB, surface BC, "
                         "128x128x192; serving: a request stream through the serving loop")
    ap.add_argument("--n", type=int, default=None, help="grid points per axis (cubic workloads)")
    ap.add_argument("--h", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--bc", default="free", choices=("free", "surface", "periodic", "wire"),
                    help="molecule workload: boundary conditions")
    ap.add_argument("--check-every", type=int, default=8,
                    help="PCG iterations per replayed graph")
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="solves of the FP64 one-at-a-time comparator (0: skip; default 2 "
                         "for charged_solute, 5 otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pass-times", action="store_true",
                    help="skip the per-pass kernel times (extra eager solves)")
    ap.add_argument("--no-extras", action="store_true",
                    help="charged_solute: skip the molecule and serving extra keys")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum wall time of the oracle sample (molecule, slab)")
    ap.add_argument("--problem", default="molecule", choices=("molecule", "manufactured"),
                    help="sc workload: the molecule, or the Gaussian test of Sec. II.C "
                         "(box 10, sigma 0.5, d0 1.7, Delta 0.3) with its analytic potential")
    ap.add_argument("--requests", type=int, default=512, help="serving: stream length")
    ap.add_argument("--max-active", type=int, default=4, help="serving: worker streams")
    ap.add_argument("--batch-slots", type=int, default=4,
                    help="serving: problems per batched launch on small grids (1: no batching)")
    ap.add_argument("--budget-frac", type=float, default=0.75,
                    help="serving: admission budget as a fraction of the distinct plans' "
                         "total resident bytes")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serving: arrival rate as a fraction of the closed-loop capacity")
    ap.add_argument("--rate", type=float, default=450.0,
                    help="serving: arrival rate in requests/s (0: --load times the closed-loop "
                         "capacity)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (10 times) and exit: the "
                         "reference for scaling FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--source-digest", action="store_true",
                    help="only print the digest of the FFT passes' sources and exit")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 10 if args.workload == "charged_solute" else 20
    if args.fp64_steps is None:
        args.fp64_steps = 2 if args.workload == "charged_solute" else 5
    return args


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_calibration(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "copies": 10}))


# the translation unit of the FFT passes (the kernels whose counters are
# recorded): their source file and every header it includes
FFT_PASS_SOURCES = ("gps_fft_fast.hip", "gps_fft_reg.h", "gps_iter.h", "gps_launch.h",
                    "gps_device.h", "gps_internal.h")


def kernel_source_digest():
    """sha256 over the FFT passes' sources (names and contents, in name order)
    and the public header they include."""
    import hashlib
    d = os.path.join(ROOT, "paper_1509_00680_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(FFT_PASS_SOURCES):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "gps.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE passes
    (scaled by a plain copy's counts), or None once the FFT passes' sources
    have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return rec["traffic_bytes_per_launch"]


def timed_solves(torch, plan, solve, steps):
    """Runs `solve` (one complete solve on `plan`) `steps` times; returns the
    wall time, per-solve latencies and the plan's info after each solve."""
    lat = []
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        st = solve(plan)
        lat.append(time.perf_counter() - s0)
        if st != 0:
            raise RuntimeError("solve failed with status %d" % st)
        infos.append(plan.info())
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat, infos


def oracle_accuracy(prob, gpu_phi, gpu_energy, workers, nonlinear_ions=None):
    """The GPU result against the oracle solved to 1e-10 (FP64, scipy.fft with
    `workers` threads).  Linear problems: the oracle's own solve of the same
    problem.  Nonlinear PB (nonlinear_ions, an oracle Electrolyte): a
    fixed-point check -- the oracle's generalized Poisson solve with the fixed
    source rho + rho^ions[phi_gpu]; at the self-consistent solution it returns
    phi_gpu itself.  Returns the figures and the oracle's timing."""
    from oracle import green, pb, pcg
    solver = green.VacuumSolver(prob.shape, prob.h, prob.bc, workers=workers)
    rho = prob.rho
    t0 = time.perf_counter()
    if nonlinear_ions is not None:
        rho = prob.rho + pb.ionic_charge(gpu_phi, nonlinear_ions,
                                         nonlinear_ions.accessibility(prob.eps))
        res = pcg.pcg_solve(rho, prob.eps, prob.h, prob.bc, tol=1e-10, solver=solver,
                            maxit=2000)
    elif prob.kind == "pb_linear":
        ions = _oracle_electrolyte(prob.ions)
        res = pb.solve_linear_pb(prob.rho, prob.eps, prob.h, prob.bc, ions, 1e-10,
                                 solver=solver)
    else:
        res = pcg.pcg_solve(rho, prob.eps, prob.h, prob.bc, tol=1e-10, solver=solver)
    dt = time.perf_counter() - t0
    e_ref = pcg.electrostatic_energy(prob.rho, res.phi, prob.h)
    return {"max_abs_dphi": float(np.abs(gpu_phi - res.phi).max()),
            "rel_energy_err": abs(gpu_energy / e_ref - 1.0),
            "oracle_tol": 1e-10, "oracle_iterations": res.iterations,
            "oracle_converged": bool(res.converged),
            "check": "fixed point: oracle PCG with the source rho + rho_ions[phi_gpu]"
            if nonlinear_ions is not None else "oracle solve of the same problem"}, \
        dt, res.iterations


def _oracle_electrolyte(d):
    from oracle import pb
    return pb.Electrolyte(d["Z"], d["c_bulk"], d["kT"], c_max=d.get("c_max"),
                          eps_bulk=d.get("eps_bulk", 78.36))


def cpu_baseline(prob, tol, min_seconds, workers, gpu_phi=None, gpu_energy=None):
    """The oracle as it stands: whole FP64 solves of the same workload at the
    bench tolerance, repeated until at least `min_seconds` have passed; then,
    with gpu_phi, the GPU result against the oracle solved to 1e-10."""
    from oracle import green, pb, pcg
    solver = green.VacuumSolver(prob.shape, prob.h, prob.bc, workers=workers)
    solves, iters = 0, 0
    t0 = time.perf_counter()
    while True:
        if prob.kind == "pb_linear":
            res = pb.solve_linear_pb(prob.rho, prob.eps, prob.h, prob.bc,
                                     _oracle_electrolyte(prob.ions), tol, solver=solver)
        else:
            res = pcg.pcg_solve(prob.rho, prob.eps, prob.h, prob.bc, tol=tol, solver=solver)
        solves += 1
        iters += res.iterations
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    out = {"value": solves / dt, "unit": "solves/s", "cores": workers, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "%d full FP64 solves of the same workload at tol %g (%d iterations "
                     "each, %.1f s, scipy.fft workers=%d)" % (solves, tol, res.iterations, dt,
                                                            workers),
           "mgridpts_iter_per_s": prob.npoints * iters / dt / 1e6}
    if gpu_phi is not None:
        out["gpu_result_vs_oracle"] = oracle_accuracy(prob, gpu_phi, gpu_energy, workers)[0]
    return out


def run_stream(torch, gps, srv, reqs, arrivals, phis):
    """Submits reqs[i] at arrivals[i] seconds (open loop) and returns the
    results and the wall time from the first submission to the last result."""
    results = [None] * len(reqs)
    pending = {}
    t0 = time.perf_counter()
    for i, (prm, rho, eps) in enumerate(reqs):
        while True:
            dt = t0 + arrivals[i] - time.perf_counter()
            if dt <= 0:
                break
            for k, t in list(pending.items()):
                r = srv.poll(t)
                if r is not None:
                    results[k] = r
                    del pending[k]
            time.sleep(min(dt, 2e-4))
        st, t = srv.submit(rho, eps, phis[i], prm["h"], prm["bc"], prm["tol"],
                           ions=prm["ions"], sync=False)
        if st != gps.GPS_OK:
            raise RuntimeError("submit failed: %s" % gps.STATUS[st])
        pending[i] = t
    for k, t in pending.items():
        results[k] = srv.wait(t)
    return results


def serving_bench(args, torch, gps, W):
    """Continuous-batching serving of a seeded request stream: open-loop
    Poisson arrivals at a fraction of the closed-loop capacity; latency is
    arrival (submission) to result ready."""
    prms, gaps = W.serving_stream_params(args.requests, seed=5)
    reqs = []
    for prm in prms:
        rho, eps = W.request_fields_torch(prm, "cuda")
        reqs.append((prm, rho, eps))
    phis = [torch.empty_like(r) for _, r, _ in reqs]
    phis64 = [torch.empty_like(r) for _, r, _ in reqs]
    torch.cuda.synchronize()
    fps = {}
    for prm in prms:
        n = prm["n"]
        tb, b, t = gps.plan_footprint((n, n, n), prm["bc"], "mixed")
        if args.batch_slots > 1 and n ** 3 <= 64 ** 3:
            b *= args.batch_slots                    # a batched plan holds batch_slots problems
        fps[(n, prm["bc"])] = (tb, b, t)
    total = sum(tb + b for tb, b, _ in fps.values())
    budget = max(int(args.budget_frac * total), max(tb + b + t for tb, b, t in fps.values()))
    npts = [prm["n"] ** 3 for prm in prms]

    def closed_loop(srv, count, out):
        t0 = time.perf_counter()
        ts = []
        for i in range(count):
            prm, rho, eps = reqs[i]
            st, t = srv.submit(rho, eps, out[i], prm["h"], prm["bc"], prm["tol"],
                               ions=prm["ions"], sync=False)
            ts.append(t)
        for t in ts:
            srv.wait(t)
        return count / (time.perf_counter() - t0)

    def summarize(results, srv):
        lat = np.array([r["done_ms"] - r["submit_ms"] for r in results])
        wait = np.array([r["start_ms"] - r["submit_ms"] for r in results])
        run = np.array([r["done_ms"] - r["start_ms"] for r in results])
        by_grid = {}
        for prm, l, w, u in zip(prms, lat, wait, run):
            by_grid.setdefault(prm["n"], []).append((l, w, u))
        per_grid = {str(n): {"requests": len(v),
                             "p50_ms": float(np.percentile([x[0] for x in v], 50)),
                             "p99_ms": float(np.percentile([x[0] for x in v], 99)),
                             "mean_wait_ms": float(np.mean([x[1] for x in v])),
                             "mean_run_ms": float(np.mean([x[2] for x in v]))}
                    for n, v in sorted(by_grid.items())}
        bad = [r["status"] for r in results if r["status"] != gps.GPS_OK]
        wall = (max(r["done_ms"] for r in results) - min(r["submit_ms"] for r in results)) / 1e3
        iters = sum(r["iterations"] for r in results)
        return {"solves_per_s": len(results) / wall, "p50_ms": float(np.percentile(lat, 50)),
                "per_grid": per_grid, "wait_p99_ms": float(np.percentile(wait, 99)),
                "p99_ms": float(np.percentile(lat, 99)), "wall_s": wall,
                "mgridpts_iter_per_s": sum(n * r["iterations"] for n, r in zip(npts, results))
                / wall / 1e6, "iterations": iters, "failed": len(bad), "stats": srv.stats()}

    # capacity: the whole stream closed-loop (every request submitted at once),
    # after one closed-loop pass that creates the plans and graphs; the open-loop
    # arrival rate is a fraction of it, so the server is not overloaded
    nreq = len(reqs)
    srv = gps.Server(budget_bytes=budget, max_active=args.max_active, precision="mixed",
                     batch_slots=args.batch_slots)
    closed_loop(srv, nreq, phis)
    capacity = closed_loop(srv, nreq, phis)
    rate = args.rate if args.rate > 0 else args.load * capacity
    arrivals = np.cumsum(gaps / rate)
    res_mixed = run_stream(torch, gps, srv, reqs, arrivals, phis)
    mixed = summarize(res_mixed, srv)
    srv.close()

    # closed-loop capacity without batched launches, for comparison
    srv1 = gps.Server(budget_bytes=budget, max_active=args.max_active, precision="mixed",
                      batch_slots=1)
    closed_loop(srv1, nreq, phis)
    capacity_unbatched = closed_loop(srv1, nreq, phis)
    srv1.close()

    srv64 = gps.Server(budget_bytes=0, max_active=1, precision="fp64")
    closed_loop(srv64, nreq, phis64)
    cap64 = closed_loop(srv64, nreq, phis64)
    res64 = run_stream(torch, gps, srv64, reqs, arrivals, phis64)
    fp64 = summarize(res64, srv64)
    srv64.close()
    fp64["closed_loop_solves_per_s"] = cap64

    dphi = 0.0
    for i, (prm, _, _) in enumerate(reqs):
        a, b = phis[i], phis64[i]
        if prm["bc"] == "periodic":
            a, b = a - a.mean(), b - b.mean()
        dphi = max(dphi, float((a - b).abs().max()))
    torch.cuda.synchronize()
    kinds = {}
    for prm in prms:
        kinds[prm["kind"]] = kinds.get(prm["kind"], 0) + 1
    return {
        "metric": "serving solves/s at 1e-6 rel. residual; p50/p99 latency (arrival to result)",
        "value": mixed["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": 2 * nreq, "ms_per_step": 1e3 / mixed["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving_stream_%d" % len(reqs), "grids": list(W.SERVING_GRIDS),
                   "box_bohr": W.SERVING_BOX, "bc": "free/surface/periodic", "kinds": kinds,
                   "seed": 5, "tol": 1e-6, "max_active": args.max_active,
                   "batch_slots": args.batch_slots,
                   "budget_bytes": budget, "distinct_plans_bytes": total,
                   "arrival_rate_per_s": rate, "closed_loop_capacity_per_s": capacity,
                   "closed_loop_capacity_unbatched_per_s": capacity_unbatched,
                   "precision": "mixed (fp32 bulk, fp64 dots/solution)"},
        "p50_ms": mixed["p50_ms"], "p99_ms": mixed["p99_ms"],
        "per_grid": mixed["per_grid"], "wait_p99_ms": mixed["wait_p99_ms"],
        "utilization": {"offered_load": rate / capacity,
                        "served_over_arrival_rate": mixed["solves_per_s"] / rate},
        "mgridpts_iter_per_s": mixed["mgridpts_iter_per_s"],
        "failed": mixed["failed"], "server": mixed["stats"],
        "fp64_one_at_a_time": dict({k: fp64[k] for k in ("solves_per_s", "p50_ms", "p99_ms",
                                                          "closed_loop_solves_per_s", "failed")},
                                   budget_bytes="unlimited", max_active=1,
                                   arrival_rate_per_s=rate, offered_load=rate / cap64),
        "max_abs_dphi_vs_fp64": dphi,
        "max_rel_energy_diff_vs_fp64": max(abs(a["energy"] / b["energy"] - 1.0)
                                           for a, b in zip(res_mixed, res64) if b["energy"]),
    }


def rigid_bench(args, torch, gps, W):
    """Rigid-cavity pipeline on one plan (Sec. IV.A): per step, the cavity and
    its analytic q (gps_rigid_cavity), the PCG solve with that q
    (gps_solve_generalized_q) and the polarization charge
    (gps_polarization_charge).  24 atoms of radius 2.2-3.0 bohr, Delta 0.5,
    on the molecule workload's grid."""
    w = W.rigid_solute(n=args.n, h=args.h, seed=args.seed, n_atoms=24, ball=6.0,
                       radii=(2.2, 3.0), delta=0.5)
    shape = w["shape"]
    rho = torch.from_numpy(w["rho"]).cuda()
    atoms = torch.from_numpy(np.ascontiguousarray(w["atoms"])).cuda()
    eps, q, phi, pol = (torch.empty_like(rho) for _ in range(4))
    plan = gps.Plan(shape, w["h"], w["bc"], precision=args.precision,
                    check_every=args.check_every)

    def step(times=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        if plan.rigid_cavity(atoms, w["delta"], w["eps0"], eps, q) != 0:
            raise RuntimeError("gps_rigid_cavity failed")
        ev[1].record()
        st = plan.solve_generalized_q(rho, eps, q, phi, args.tol)
        if st != 0:
            raise RuntimeError("solve failed with status %d" % st)
        ev[2].record()
        if plan.polarization_charge(rho, eps, phi, pol) != 0:
            raise RuntimeError("gps_polarization_charge failed")
        ev[3].record()
        if times is not None:
            torch.cuda.synchronize()
            times.append([ev[i].elapsed_time(ev[i + 1]) for i in range(3)])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = []
    for _ in range(args.steps):
        step(times)
    tm = np.mean(np.array(times), axis=0)
    info = plan.info()
    npts = int(np.prod(shape))
    pol_bytes = 32.0 * npts          # eps, phi, rho read, rho_pol written (FP64)
    total_pol = float(pol.sum().item()) * w["h"] ** 3
    qsum = float(np.sum(w["rho"])) * w["h"] ** 3
    return {
        "metric": "rigid-cavity pipeline steps/s (cavity + analytic q, PCG at 1e-6, "
                  "polarization charge)",
        "value": args.steps / wall, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": w["name"] + "_rigid_free", "grid": list(shape), "h": w["h"],
                   "n_atoms": 24, "delta": w["delta"], "tol": args.tol,
                   "precision": args.precision},
        "iters_per_solve": info["iterations"],
        "event_ms": {"rigid_cavity": tm[0], "solve": tm[1], "polarization": tm[2]},
        "polarization_gbs_event": pol_bytes / (tm[2] * 1e-3) / 1e9,
        "atom_points_per_s_event": 24.0 * npts / (tm[0] * 1e-3),
        "polarization_total": total_pol, "solute_charge": qsum,
    }


def sc_bench(args, torch, gps, W):
    """Algorithm SC (mixing 0.6) and PSD on the molecule workload, against
    Algorithm PCG on the same plan (Sec. II.A vs II.B): iterations, solves/s
    and time per iteration at the same tolerance (SC and PSD measure their
    own residuals, ||rho_iter_{k+1} - rho_iter_k|| / ||rho|| and ||r/eps||)."""
    exact = None
    if args.problem == "manufactured":
        prob, exact = W.manufactured_gaussian(args.n, box=10.0, sigma=0.5, d0=1.7, delta=0.3)
        name = "manufactured%d" % args.n
    else:
        prob = W.molecule(args.n, args.h, seed=args.seed, bc=args.bc)
        name = "molecule%d_sccs_%s" % (args.n, args.bc)
    rho = torch.from_numpy(prob.rho).cuda()
    eps = torch.from_numpy(prob.eps).cuda()
    phi = torch.empty_like(rho)
    plan = gps.Plan(prob.shape, prob.h, prob.bc, precision=args.precision, maxit=5000,
                    check_every=args.check_every)
    out = {}
    for meth, run in (("pcg", lambda: plan.solve_generalized(rho, eps, phi, args.tol)),
                      ("sc", lambda: plan.solve_sc(rho, eps, phi, args.tol, "sc", 0.6)),
                      ("psd_weighted",
                       lambda: plan.solve_sc(rho, eps, phi, args.tol, "psd_weighted"))):
        run()
        torch.cuda.synchronize()
        reps = max(1, args.steps // (1 if meth == "pcg" else 4))
        t0 = time.perf_counter()
        for _ in range(reps):
            st = run()
            if st != 0:
                raise RuntimeError("%s failed with status %d" % (meth, st))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        it = plan.info()["iterations"]
        out[meth] = {"solves_per_s": 1.0 / dt, "iterations": it, "ms_per_solve": dt * 1e3,
                     "us_per_iteration": dt * 1e6 / max(1, it), "energy": plan.info()["energy"]}
        if exact is not None:
            out[meth]["max_error_vs_analytic"] = float(np.abs(phi.cpu().numpy() - exact).max())
    # PSD with Algorithm PCG's own step (beta = 0): reported with its status,
    # since it does not contract on this discretization
    p200 = gps.Plan(prob.shape, prob.h, prob.bc, precision=args.precision, maxit=200)
    st = p200.solve_sc(rho, eps, phi, args.tol, "psd")
    out["psd"] = {"status": gps.STATUS[st], "iterations": p200.info()["iterations"],
                  "rel_residual": p200.info()["rel_residual"]}
    p200.close()
    return {
        "metric": "SC and PSD against PCG: solves/s at the same tolerance",
        "value": out["sc"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": out["sc"]["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": name, "tol": args.tol, "precision": args.precision, "eta": 0.6},
        "methods": out,
    }


def solve_fn(prob):
    """A closure running one complete solve of `prob` on a plan (generalized
    Poisson, or Poisson-Boltzmann when the problem has an electrolyte)."""
    def solve(plan, rho, eps, phi, tol):
        if prob.ions is None:
            return plan.solve_generalized(rho, eps, phi, tol)
        return plan.solve_pb(rho, eps, prob.ions, phi, tol)
    return solve


def pcg_line(args, torch, gps, W, prob, name, steps, warmup, cpu=True, pass_times=True):
    """The bench line of one PCG / PB workload: solves/s, Mgridpts*iter/s over
    all PCG iterations, latency, roofline of the z pass, per-pass times, the
    FP64 one-at-a-time comparator, the oracle's accuracy check and timing."""
    rho = torch.from_numpy(prob.rho).cuda()
    eps = torch.from_numpy(prob.eps).cuda()
    phi = torch.empty_like(rho)
    run = solve_fn(prob)
    nonlinear = prob.kind == "pb_nonlinear"
    plan = gps.Plan(prob.shape, prob.h, prob.bc, precision=args.precision,
                    check_every=args.check_every)

    def solve(pl):
        return run(pl, rho, eps, phi, args.tol)

    for _ in range(warmup):
        solve(plan)
    # timed region (iterations replayed as HIP graphs)
    wall, lat, infos = timed_solves(torch, plan, solve, steps)
    iters = [i["iterations"] for i in infos]
    info = infos[-1]
    phi_gpu = phi.cpu().numpy()             # the last timed solve's potential
    # dominant pass: every launch bracketed by HIP events on the solve stream
    # (kernels launched one by one while timed)
    plan.set_timing("zconv")
    timed_solves(torch, plan, solve, 1 if nonlinear else max(3, steps // 4))
    tz = plan.timing()
    plan.set_timing(None)
    avg_ms = tz["total_ms"] / max(1, tz["launches"])
    achieved = tz["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0

    pass_ms = {}
    if pass_times:
        for k in PASSES:
            plan.set_timing(k)
            timed_solves(torch, plan, solve, 1 if nonlinear else 2)
            t = plan.timing()
            us = 1e3 * t["total_ms"] / max(1, t["launches"])
            pass_ms[k] = {"avg_us": us, "bytes_per_launch": t["bytes_per_launch"],
                          "gbs": t["bytes_per_launch"] / (us * 1e-6) / 1e9 if us > 0 else 0.0}
        plan.set_timing(None)
    plan.close()

    fp64 = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        p64 = gps.Plan(prob.shape, prob.h, prob.bc, precision="fp64",
                       check_every=args.check_every)
        solve(p64)
        w64, l64, i64 = timed_solves(torch, p64, solve, args.fp64_steps)
        fp64 = {"solves_per_s": args.fp64_steps / w64,
                "p99_ms": float(np.percentile(np.array(l64) * 1e3, 99)),
                "iters_per_solve": float(np.mean([i["iterations"] for i in i64])),
                "max_abs_dphi_vs_this": float(np.abs(phi.cpu().numpy() - phi_gpu).max()),
                "rel_energy_diff_vs_this": abs(info["energy"] / i64[-1]["energy"] - 1.0)}
        if nonlinear:
            fp64["outer_per_solve"] = float(np.mean([i["outer_iterations"] for i in i64]))
        p64.close()

    lat_ms = np.array(lat) * 1e3
    traffic_file = "traffic_zpass_%s_%s.json" % (name, args.precision)
    out = {
        "value": steps / wall,
        "unit": "solves/s",
        "ms_per_step": wall / steps * 1e3,
        "mgridpts_iter_per_s": prob.npoints * sum(iters) / wall / 1e6,
        "iters_per_solve": float(np.mean(iters)),
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "energy": info["energy"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(traffic_file),
                     "kernel": "z pass (forward FFT, Green's spectrum, inverse FFT)",
                     "avg_us": avg_ms * 1e3, "bytes_per_launch": tz["bytes_per_launch"],
                     "launches": tz["launches"]},
        "fp64_one_at_a_time": fp64,
    }
    if nonlinear:
        out["outer_per_solve"] = float(np.mean([i["outer_iterations"] for i in infos]))
        out["outer_residual"] = info["outer_residual"]
    if pass_ms:
        out["passes"] = pass_ms
    if cpu and not args.no_cpu_baseline:
        workers = min(16, os.cpu_count() or 1)
        if nonlinear:
            # the oracle's sample is the accuracy check itself: one FP64 PCG solve
            # at 160^3 to 1e-10, timed per iteration and scaled to whole nonlinear
            # solves with the FP64 path's inner iteration count
            acc, dt, it = oracle_accuracy(prob, phi_gpu, info["energy"], workers,
                                          nonlinear_ions=_oracle_electrolyte(prob.ions))
            per_solve = fp64["iters_per_solve"] if fp64 else float(np.mean(iters))
            rate = it / dt
            out["cpu_baseline"] = {
                "value": rate / per_solve, "unit": "solves/s", "cores": workers,
                "kind": "oracle", "cpu_model": cpu_model(),
                "sample": "one FP64 oracle PCG solve of the %s generalized Poisson problem "
                          "with the source rho + rho_ions[phi_gpu], to 1e-10 (%d iterations, "
                          "%.1f s, scipy.fft workers=%d); solves/s = iterations/s over the "
                          "%.0f inner iterations of one FP64 nonlinear solve"
                          % ("x".join(map(str, prob.shape)), it, dt, workers, per_solve),
                "mgridpts_iter_per_s": prob.npoints * rate / 1e6,
                "gpu_result_vs_oracle": acc}
        else:
            out["cpu_baseline"] = cpu_baseline(prob, args.tol, args.cpu_seconds, workers,
                                               gpu_phi=phi_gpu, gpu_energy=info["energy"])
    return out


def refine_bench(args, torch, gps, W):
    """Mixed precision with FP64 true-residual refinement, and warm starts, on
    the molecule workload: iterations, time per solve and the distance to an
    FP64 GPU solve at 1e-11 (the reference; FP64 and the oracle agree to 1e-13
    at this size, test_gpu_configs)."""
    prob = W.molecule(args.n or 96, args.h, seed=2 if args.seed is None else args.seed)
    other = W.molecule(args.n or 96, args.h, seed=3)
    rho = torch.from_numpy(prob.rho).cuda()
    rho2 = torch.from_numpy(prob.rho + 0.02 * other.rho).cuda()
    eps = torch.from_numpy(prob.eps).cuda()
    phi, ref, ref2 = torch.empty_like(rho), torch.empty_like(rho), torch.empty_like(rho)
    p64 = gps.Plan(prob.shape, prob.h, prob.bc, precision="fp64", maxit=5000)
    for r, out in ((rho, ref), (rho2, ref2)):
        if p64.solve_generalized(r, eps, out, 1e-11) != 0:
            raise RuntimeError("FP64 reference solve failed")
    e_ref = p64.info()["energy"]
    p64.solve_generalized(rho, eps, ref, 1e-11)
    e_ref = p64.info()["energy"]
    p64.close()
    rows = []

    def run(label, tol, refine, reps=5):
        pl = gps.Plan(prob.shape, prob.h, prob.bc, precision="mixed", maxit=5000,
                      check_every=args.check_every, refine_every=refine)
        pl.solve_generalized(rho, eps, phi, tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if pl.solve_generalized(rho, eps, phi, tol) != 0:
                raise RuntimeError(label + " failed")
        torch.cuda.synchronize()
        info = pl.info()
        rows.append({"mode": label, "tol": tol, "iterations": info["iterations"],
                     "ms_per_solve": (time.perf_counter() - t0) / reps * 1e3,
                     "max_abs_dphi": float((phi - ref).abs().max()),
                     "rel_energy_err": abs(info["energy"] / e_ref - 1.0)})
        pl.close()

    run("mixed", 1e-6, 0)
    run("mixed, refine every 20", 1e-6, 20)
    run("mixed", 1e-9, 0)
    run("mixed, refine every 20", 1e-9, 20)
    # warm start on one plan and dielectric: cold, the same rho again, a perturbed rho
    pl = gps.Plan(prob.shape, prob.h, prob.bc, precision="mixed", check_every=args.check_every,
                  warm_start=True)
    warm = []
    for label, r, rf in (("cold", rho, ref), ("same rho", rho, ref), ("rho + 2% of another solute",
                                                                     rho2, ref2)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if pl.solve_generalized(r, eps, phi, 1e-6) != 0:
            raise RuntimeError("warm start " + label)
        torch.cuda.synchronize()
        warm.append({"solve": label, "iterations": pl.info()["iterations"],
                     "ms": (time.perf_counter() - t0) * 1e3,
                     "max_abs_dphi": float((phi - rf).abs().max())})
    pl.close()
    return {
        "metric": "mixed-precision refinement and warm start: iterations, ms per solve and "
                  "distance to the FP64 solve",
        "value": 1e3 / rows[1]["ms_per_solve"], "unit": "solves/s (mixed, refine every 20, tol 1e-6)",
        "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": rows[1]["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "molecule%d_sccs_free_refine" % prob.shape[0],
                   "reference": "FP64 GPU solve at 1e-11"},
        "refinement": rows, "warm_start": warm,
    }


def micro_bench(args, torch):
    """Measurements behind the FFT design (libgps_micro.so): the FP32 issue
    rate of the 16-point register codelet, the same DFT as a dense real GEMM on
    the matrix cores (checked against numpy's FFT, then timed with register
    operands only: an upper bound for any MFMA form of the stage), and the
    floor of a 5-read / 2-write pointwise pass at 96^3 and 160^3 points."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1509_00680_amd", "libgps_micro.so"))
    vp, ci, cl = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong
    lib.micro_codelet16.argtypes = [ci, ci, vp, vp]
    lib.micro_mfma_dft16_check.argtypes = [vp, vp, vp]
    lib.micro_mfma_dft16_rate.argtypes = [ci, ci, vp, vp]
    lib.micro_stream5.argtypes = [cl, vp, vp, vp, vp, vp, vp, vp, vp]
    stream = vp(torch.cuda.current_stream().cuda_stream)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    # the GEMM form computes the DFT
    rng = np.random.default_rng(0)
    xh = rng.normal(size=(32, 16)).astype(np.float32)
    x = torch.from_numpy(xh).cuda()
    y = torch.empty_like(x)
    if lib.micro_mfma_dft16_check(vp(x.data_ptr()), vp(y.data_ptr()), stream) != 0:
        raise RuntimeError("micro_mfma_dft16_check launch failed")
    z = np.fft.fft(xh[:16].astype(np.float64) + 1j * xh[16:].astype(np.float64), axis=0)
    ref = np.concatenate([z.real, z.imag])
    mfma_err = float(np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max())

    blocks, reps = 4096, 400
    out = torch.empty(blocks * 256, device="cuda")
    t_cod = timed(lambda: lib.micro_codelet16(blocks, reps, vp(out.data_ptr()), stream), 5)
    t_mf = timed(lambda: lib.micro_mfma_dft16_rate(blocks, reps, vp(out.data_ptr()), stream), 5)
    lanes = blocks * 256
    cod_rate = lanes * reps / t_cod                  # pencils/s, one pencil per lane
    waves = lanes // 64
    mf_inst = waves * 16 * reps / t_mf               # MFMA instructions/s
    mf_rate = mf_inst                                # 16 MFMAs per 16 pencils

    streams = {}
    for n in (96, 160):
        npts = n ** 3
        bufs = [torch.rand(npts, device="cuda") for _ in range(7)]
        t = timed(lambda: lib.micro_stream5(npts, *[vp(b.data_ptr()) for b in bufs], stream), 20)
        streams["%d^3" % n] = {"bytes": 28 * npts, "us": t * 1e6, "gbs": 28 * npts / t / 1e9}
    return {
        "metric": "FFT design micro-benchmarks: 16-point DFT per second as register codelet "
                  "and as MFMA GEMM; pointwise-pass floor",
        "value": cod_rate / 1e9, "unit": "G 16-point DFTs/s (register codelet)",
        "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": t_cod * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "micro_fft_design", "codelet_lanes": lanes, "reps": reps,
                   "mfma": "v_mfma_f32_16x16x4_f32, 16 per 16 pencils (32x32 real DFT matrix)"},
        "codelet_dft16_per_s": cod_rate,
        "mfma_dft16_per_s_upper_bound": mf_rate,
        "mfma_tflops": mf_inst * 2048 / 1e12,
        "codelet_over_mfma": cod_rate / mf_rate,
        "mfma_dft_check_max_rel_err": mfma_err,
        "pointwise_5r2w": streams,
    }


def main():
    args = parse()
    if args.source_digest:
        print(kernel_source_digest())
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(one GPU per process; requests would shard one plan per GPU)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    from paper_1509_00680_amd import gps, workloads as W
    if args.workload == "serving":
        print(json.dumps(serving_bench(args, torch, gps, W)))
        return
    if args.workload == "micro":
        print(json.dumps(micro_bench(args, torch)))
        return
    if args.workload == "refine":
        print(json.dumps(refine_bench(args, torch, gps, W)))
        return
    if args.workload == "rigid":
        args.n = args.n or 96
        args.seed = 2 if args.seed is None else args.seed
        print(json.dumps(rigid_bench(args, torch, gps, W)))
        return
    if args.workload == "sc":
        args.n = args.n or 96
        args.seed = 2 if args.seed is None else args.seed
        print(json.dumps(sc_bench(args, torch, gps, W)))
        return

    if args.workload == "charged_solute":
        n = args.n or 160
        seed = 4 if args.seed is None else args.seed
        prob = W.charged_solute_mpb(n=n, h=args.h, seed=seed, tol=args.tol)
        name = "charged_solute%d_mpb_free" % n
        config = {"workload": name, "grid": list(prob.shape), "h": prob.h, "bc": "free",
                  "n_charges": 48, "net_charge": 4.0, "seed": seed,
                  "electrolyte": "1:1, 1 M, steric (p 0.74, R 3 A), gamma = (eps-1)/(eps0-1)",
                  "algorithm": "SCPBimproved, eta %g" % prob.ions["eta"],
                  "tol": args.tol}
        metric = ("PCG solves/s and Mgridpts\u00b7iter/s at 1e-6 rel. residual; p50/p99 "
                  "latency")
    elif args.workload == "slab":
        prob = W.slab(tol=args.tol)
        name = "slab128x128x192_surface"
        config = {"workload": name, "grid": list(prob.shape), "h": prob.h, "bc": "surface",
                  "n_charges": 64, "seed": 3, "electrolyte": "linear PB, Debye length 10 bohr",
                  "tol": args.tol}
        metric = "PCG solves/s and Mgridpts\u00b7iter/s at 1e-6 rel. residual; p50/p99 latency"
    else:
        n = args.n or 96
        seed = 2 if args.seed is None else args.seed
        prob = W.molecule(n, args.h, seed=seed, bc=args.bc, tol=args.tol)
        name = "molecule%d_sccs_%s" % (n, args.bc)
        config = {"workload": name, "grid": list(prob.shape), "h": prob.h, "bc": prob.bc,
                  "n_charges": 24, "seed": seed, "tol": args.tol}
        metric = "PCG solves/s and Mgridpts\u00b7iter/s at 1e-6 rel. residual; p50/p99 latency"
    config["precision"] = args.precision + (" (fp32 bulk, fp64 dots/solution)"
                                            if args.precision == "mixed" else "")
    line = pcg_line(args, torch, gps, W, prob, name, args.steps, args.warmup,
                    pass_times=not args.no_pass_times)
    out = {"metric": json.loads('"%s"' % metric), "value": line.pop("value"),
           "unit": line.pop("unit"), "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": line.pop("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
           "config": config}
    out.update(line)
    if args.workload == "charged_solute" and not args.no_extras:
        # the molecule 96^3 line and the serving stream, as extra keys
        mol = W.molecule(96, 0.3, seed=2, tol=args.tol)
        m = pcg_line(args, torch, gps, W, mol, "molecule96_sccs_free", 20, 3, cpu=False,
                     pass_times=False)
        out["molecule96_sccs_free"] = {k: m[k] for k in (
            "value", "unit", "mgridpts_iter_per_s", "iters_per_solve", "p50_ms", "p99_ms",
            "fp64_one_at_a_time")}
        out["molecule96_sccs_free"]["roofline_frac"] = m["roofline"]["frac"]
        sv = serving_bench(args, torch, gps, W)
        out["serving_stream512"] = {k: sv[k] for k in (
            "value", "unit", "p50_ms", "p99_ms", "utilization", "fp64_one_at_a_time",
            "max_abs_dphi_vs_fp64")}
        out["serving_stream512"]["arrival_rate_per_s"] = sv["config"]["arrival_rate_per_s"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
