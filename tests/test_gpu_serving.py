"""Serving (gps_server_*): a stream of independent requests of different grids,
boundary conditions and kinds, admitted by device footprint and run
concurrently on several streams, small grids in continuous batches (several
problems per launch, joining and leaving between graph replays).  Each result
must equal, bit for bit, the same request solved alone on a fresh plan;
served requests, batched ones included, are checked against the FP64 oracle;
footprints agree with what plans actually hold."""
import numpy as np
import pytest

from oracle import pb, pcg
from paper_1509_00680_amd import gps
from paper_1509_00680_amd import workloads as W
from gpu_util import dev, host, empty, plan, oracle_ions, require_gpu

pytestmark = pytest.mark.gpu

GRIDS = (16, 24, 32)
BOX = 9.6


def _requests(n, seed):
    prms, _ = W.serving_stream_params(n, seed=seed, grids=GRIDS, box=BOX)
    out = []
    for prm in prms:
        prob = W.request_problem(prm)
        out.append((prob, dev(prob.rho), dev(prob.eps)))
    return out


def _solve_alone(prob, rho, eps, precision="mixed"):
    p = plan(prob.shape, prob.h, prob.bc, precision)
    phi = empty(prob.shape)
    if prob.ions is None:
        st = p.solve_generalized(rho, eps, phi, prob.tol)
    else:
        st = p.solve_pb(rho, eps, prob.ions, phi, prob.tol)
    info = p.info()
    p.close()
    return st, phi, info


@pytest.mark.parametrize("bc", ["free", "surface", "periodic", "wire"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_footprint_matches_plan_bytes(bc, precision):
    require_gpu()
    prob = W.molecule(24, 0.4, seed=3, n_atoms=6, ball=2.0, bc=bc)
    p = plan(prob.shape, prob.h, bc, precision)
    phi = empty(prob.shape)
    print("footprint", bc, precision, flush=True)
    assert p.solve_generalized(dev(prob.rho), dev(prob.eps), phi, 1e-6) == gps.GPS_OK
    tables, buffers, _ = gps.plan_footprint(prob.shape, bc, precision)
    assert p.device_bytes() == tables + buffers
    phi0 = host(phi)
    p.release_buffers()
    assert p.device_bytes() == tables
    # the buffers come back on the next solve, with the same result
    assert p.solve_generalized(dev(prob.rho), dev(prob.eps), phi, 1e-6) == gps.GPS_OK
    assert p.device_bytes() == tables + buffers
    assert np.array_equal(host(phi), phi0)
    if bc != "periodic":
        ions = W.electrolyte_1to1(W.debye_concentration(3.0), eta=0.3)
        assert p.solve_pb(dev(prob.rho * 1e-3), dev(prob.eps), ions, phi, 1e-5) == gps.GPS_OK
        _, buffers_nl, _ = gps.plan_footprint(prob.shape, bc, precision, nonlinear_pb=True)
        assert p.device_bytes() == tables + buffers_nl


def _mix(reqs, srv):
    torch = require_gpu()
    phis, tickets = [], []
    for prob, rho, eps in reqs:
        phi = torch.full(prob.shape, float("nan"), dtype=torch.float64, device="cuda")
        st, t = srv.submit(rho, eps, phi, prob.h, prob.bc, prob.tol, ions=prob.ions)
        assert st == gps.GPS_OK
        phis.append(phi)
        tickets.append(t)
    return phis, [srv.wait(t) for t in tickets]


def _check_alone(reqs, phis, results):
    torch = require_gpu()
    for (prob, rho, eps), phi, res in zip(reqs, phis, results):
        print("alone", prob.name, flush=True)
        st, phi1, info = _solve_alone(prob, rho, eps)
        assert res["status"] == st == gps.GPS_OK, (prob.name, res, st)
        assert res["iterations"] == info["iterations"]
        assert res["energy"] == info["energy"]
        assert torch.equal(phi, phi1), prob.name
        assert res["submit_ms"] <= res["start_ms"] <= res["done_ms"]


@pytest.mark.parametrize("slots", [1, 4])
def test_mix_equals_alone_bitwise(slots):
    torch = require_gpu()
    reqs = _requests(18, seed=7)
    fp = {(p.shape, p.bc): gps.plan_footprint(p.shape, p.bc, "mixed") for p, _, _ in reqs}
    fp = {k: (tb, b * slots, t) for k, (tb, b, t) in fp.items()}
    # every request fits alone, the distinct plans together do not
    budget = (max(tb + b + t for tb, b, t in fp.values())
              + sum(tb + b for tb, b, _ in fp.values()) // 4)
    assert sum(tb + b for tb, b, _ in fp.values()) > budget
    srv = gps.Server(budget_bytes=budget, max_active=4, precision="mixed", batch_slots=slots)
    print("serving mix of", len(reqs), "requests, budget", budget, "slots", slots, flush=True)
    phis, results = _mix(reqs, srv)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(reqs)
    assert stats["max_in_flight"] >= 2
    assert stats["bytes_peak"] <= budget
    assert stats["plans_evicted"] + stats["buffers_released"] >= 1   # the budget binds
    assert stats["batched"] == (len(reqs) if slots > 1 else 0)
    _check_alone(reqs, phis, results)


def test_batched_stream_joins_and_matches_oracle():
    # many requests on few plans: batches fill, requests join freed slots, and
    # each result equals its solve alone (bitwise) and the oracle (1e-5 Ha/e,
    # relative energy 1e-6)
    require_gpu()
    prms, _ = W.serving_stream_params(24, seed=11, grids=(24,), box=BOX)
    for i, prm in enumerate(prms):
        prm["bc"] = ("free", "surface")[i % 2]
        prm["kind"], prm["ions"] = "gpe", None
    reqs = []
    for prm in prms:
        prob = W.request_problem(prm)
        reqs.append((prob, dev(prob.rho), dev(prob.eps)))
    srv = gps.Server(max_active=2, precision="mixed", batch_slots=4)
    print("batched stream of", len(reqs), "requests", flush=True)
    phis, results = _mix(reqs, srv)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == stats["batched"] == len(reqs)
    assert stats["max_batch"] == 4
    assert stats["plans_created"] <= 2 * 2
    _check_alone(reqs, phis, results)
    for (prob, _, _), phi, res in list(zip(reqs, phis, results))[::6]:
        print("oracle", prob.name, flush=True)
        ref = pcg.pcg_solve(prob.rho, prob.eps, prob.h, prob.bc, tol=1e-10)
        assert np.abs(host(phi) - ref.phi).max() <= 1e-5
        e_ref = pcg.electrostatic_energy(prob.rho, ref.phi, prob.h)
        assert abs(res["energy"] / e_ref - 1.0) <= 1e-6


def test_bench_stream_sample_matches_oracle():
    # the stream the serving bench replays (512 requests, seed 5, grids 32-128
    # in a 19.2-bohr box): its requests of at most 48^3 among the first 60 (both
    # kinds, the three BCs), served in batches under the mixed server, each
    # against the oracle at 1e-10 -- max |dphi| <= 1e-5 Ha/e and relative
    # energy 1e-6 (periodic GPe: up to the constant)
    require_gpu()
    from oracle import pb
    from gpu_util import oracle_ions
    prms, _ = W.serving_stream_params(512, seed=5)
    picked = [prm for prm in prms[:60] if prm["n"] <= 48]
    reqs = []
    for prm in picked:
        prob = W.request_problem(prm)
        reqs.append((prob, dev(prob.rho), dev(prob.eps)))
    kinds = {(prob.bc, prob.kind) for prob, _, _ in reqs}
    assert len(reqs) >= 10 and len(kinds) >= 5, kinds
    srv = gps.Server(max_active=4, precision="mixed", batch_slots=4)
    print("bench stream sample of", len(reqs), "requests", flush=True)
    phis, results = _mix(reqs, srv)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(reqs) and stats["batched"] >= 1
    worst_phi = worst_e = 0.0
    for (prob, _, _), phi, res in zip(reqs, phis, results):
        print("oracle", prob.name, flush=True)
        assert res["status"] == gps.GPS_OK, (prob.name, res)
        if prob.ions is None:
            ref = pcg.pcg_solve(prob.rho, prob.eps, prob.h, prob.bc, tol=1e-10).phi
        else:
            ref = pb.solve_linear_pb(prob.rho, prob.eps, prob.h, prob.bc, oracle_ions(prob.ions),
                                     1e-10).phi
        got = host(phi)
        if prob.bc == "periodic" and prob.ions is None:
            got, ref = got - got.mean(), ref - ref.mean()
        worst_phi = max(worst_phi, float(np.abs(got - ref).max()))
        e_ref = pcg.electrostatic_energy(prob.rho, ref, prob.h)
        worst_e = max(worst_e, abs(res["energy"] / e_ref - 1.0))
    print("served vs oracle: max |dphi| %.2e, max rel dE %.2e" % (worst_phi, worst_e), flush=True)
    assert worst_phi <= 1e-5 and worst_e <= 1e-6


def test_served_request_matches_oracle():
    require_gpu()
    prm = W.serving_params(np.random.default_rng(3), grids=(24,), box=BOX)
    prm["bc"], prm["kind"], prm["ions"] = "periodic", "gpe", None
    prob = W.request_problem(prm)
    ref = pcg.pcg_solve(prob.rho, prob.eps, prob.h, "periodic", tol=1e-10)
    srv = gps.Server(max_active=2, precision="mixed")
    phi = empty(prob.shape)
    print("served periodic request vs oracle", flush=True)
    st, t = srv.submit(dev(prob.rho), dev(prob.eps), phi, prob.h, prob.bc, 1e-6)
    assert st == gps.GPS_OK
    res = srv.wait(t)
    srv.close()
    assert res["status"] == gps.GPS_OK
    got = host(phi)
    # periodic GPe: unique up to a constant
    d = (got - got.mean()) - (ref.phi - ref.phi.mean())
    assert np.abs(d).max() <= 1e-5
    e_ref = pcg.electrostatic_energy(prob.rho, ref.phi, prob.h)
    assert abs(res["energy"] / e_ref - 1.0) <= 1e-6


def test_served_nonlinear_pb_matches_oracle():
    # a nonlinear PB request (Algorithm SCPBimproved, steric ions) served beside a
    # batchable GPe request, both against the oracle
    require_gpu()
    prob = W.charged_solute_mpb(n=24, h=0.5, n_atoms=8, ball=2.0, net_charge=1.0,
                                molar=0.1, steric=True)
    ref = pb.scpb_improved(prob.rho, prob.eps, prob.h, "free", oracle_ions(prob.ions), 1e-9,
                           eta=prob.ions["eta"])
    assert ref.converged
    small = W.molecule(16, 0.5, seed=6, n_atoms=4, ball=2.0)
    ref_small = pcg.pcg_solve(small.rho, small.eps, small.h, "free", tol=1e-10)
    srv = gps.Server(max_active=2, precision="mixed")
    phi, phi_small = empty(prob.shape), empty(small.shape)
    print("served nonlinear pb beside a gpe request", flush=True)
    st, t = srv.submit(dev(prob.rho), dev(prob.eps), phi, prob.h, "free", 1e-6, ions=prob.ions)
    assert st == gps.GPS_OK
    st, t_small = srv.submit(dev(small.rho), dev(small.eps), phi_small, small.h, "free", 1e-6)
    assert st == gps.GPS_OK
    res, res_small = srv.wait(t), srv.wait(t_small)
    srv.close()
    assert res["status"] == gps.GPS_OK and res_small["status"] == gps.GPS_OK
    assert res["outer_iterations"] > 2
    assert np.abs(host(phi) - ref.phi).max() <= 1e-5
    assert np.abs(host(phi_small) - ref_small.phi).max() <= 1e-5
    e_ref = pcg.electrostatic_energy(small.rho, ref_small.phi, small.h)
    assert abs(res_small["energy"] / e_ref - 1.0) <= 1e-6


def test_server_errors_and_polling():
    torch = require_gpu()
    prob = W.molecule(16, 0.5, seed=1, n_atoms=4, ball=2.0)
    rho, eps = dev(prob.rho), dev(prob.eps)
    small = gps.plan_footprint((16, 16, 16), "free", "mixed")
    srv = gps.Server(budget_bytes=sum(small), max_active=1, precision="mixed", batch_slots=1)
    big = torch.zeros((32, 32, 32), dtype=torch.float64, device="cuda")
    st, _ = srv.submit(big, big, big.clone(), 0.5, "free", 1e-6)
    assert st == gps.GPS_E_NOMEM                    # can never fit the budget
    phi = empty(prob.shape)
    st, t = srv.submit(rho, eps, phi, prob.h, "free", 1e-6)
    assert st == gps.GPS_OK
    # a grid whose padded FFT length (22) has the factor 11: failed in the result
    odd = torch.ones((11, 11, 11), dtype=torch.float64, device="cuda")
    st, t_bad = srv.submit(odd * 0.0, odd, odd.clone(), 0.5, "free", 1e-6)
    assert st == gps.GPS_OK
    res = srv.wait(t)
    assert res["status"] == gps.GPS_OK
    assert srv.wait(t_bad)["status"] == gps.GPS_E_UNSUPPORTED
    with pytest.raises(gps.GPSError):
        srv.poll(t)                                 # released ticket
    stats = srv.stats()
    srv.close()
    assert stats["submitted"] == stats["completed"] == 2


def test_warm_start_cache_by_eps_key():
    # requests that name the same dielectric (eps_key) reuse the plan's cached
    # iterate: a re-solve of the same rho needs a few iterations, a perturbed
    # rho fewer than cold; results match the oracle; another key starts cold
    require_gpu()
    prob = W.molecule(32, 0.4, seed=5, n_atoms=8, ball=2.0)
    other = W.molecule(32, 0.4, seed=6, n_atoms=8, ball=2.0)
    rho, eps = dev(prob.rho), dev(prob.eps)
    rho2 = dev(prob.rho + 0.02 * other.rho)
    srv = gps.Server(max_active=1, precision="mixed")
    out = []
    print("warm-start cache", flush=True)
    for r, key in ((rho, 7), (rho, 7), (rho2, 7), (rho, 8)):
        phi = empty(prob.shape)
        st, t = srv.submit(r, eps, phi, prob.h, "free", 1e-6, eps_key=key)
        assert st == gps.GPS_OK
        out.append((srv.wait(t), phi))
    srv.close()
    (c0, p0), (w1, p1), (w2, p2), (c3, p3) = out
    assert [x["status"] for x, _ in out] == [gps.GPS_OK] * 4
    assert [x["warm_started"] for x, _ in out] == [0, 1, 1, 0]
    print("  iterations cold %d, same rho %d, perturbed %d, other key %d"
          % (c0["iterations"], w1["iterations"], w2["iterations"], c3["iterations"]))
    assert w1["iterations"] <= c0["iterations"] // 4
    assert w2["iterations"] < c0["iterations"]
    ref = pcg.pcg_solve(prob.rho, prob.eps, prob.h, "free", tol=1e-10)
    ref2 = pcg.pcg_solve(prob.rho + 0.02 * other.rho, prob.eps, prob.h, "free", tol=1e-10)
    for phi, r in ((p0, ref), (p1, ref), (p2, ref2), (p3, ref)):
        assert np.abs(host(phi) - r.phi).max() <= 1e-5
