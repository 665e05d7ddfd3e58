"""Serving loop on the GPU: requests of mixed lattices, boundary types,
kappas, precisions and rhs counts run concurrently through lqcd_submit /
lqcd_poll; every result must equal (bitwise) the same solve run alone with
lqcd_solve, and meet the tolerance against the oracle."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_16994_amd import inputs, lqcd

pytestmark = pytest.mark.gpu

TH_P = (1, 1, 1, -1)
TH_O = (1, 1, 1, 1)
LATS = [((8, 8, 8, 8), lqcd.BC_PERIODIC, TH_P, 31), ((8, 8, 8, 16), lqcd.BC_OPEN, TH_O, 32),
        ((16, 16, 16, 32), lqcd.BC_PERIODIC, TH_P, 33)]


def _wait(srv, tickets, timeout=120.0):
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout
        time.sleep(0.002)
    return out


def test_mixed_requests_match_alone():
    """Ten requests of mixed lattices, boundary types, kappas, inner
    precisions and rhs counts: four at once, then one every 20 ms while the
    first ones run.  The device work of requests overlaps in time, requests
    arrive and are admitted while others are on the GPU, every result is
    bitwise the same solve run alone, and every column meets 1e-10 by the
    oracle's residual (all lattices, 16^3x32 included)."""
    pm = lqcd.PM_F64 | lqcd.PM_F32
    fields = [inputs.gauge_field(L, 0.2, seed=sd, bc=bc) for L, bc, th, sd in LATS]
    srv = lqcd.Server(8 << 30, max_streams=4)
    gids = [srv.add_gauge(L, bc, th, U, pm) for (L, bc, th, _), U in zip(LATS, fields)]
    # kernels tuned before serving (requests never tune)
    srv.warmup(gids[2], lqcd.F32, 3)
    srv.warmup(gids[0], lqcd.F64, 1)
    assert lqcd.tune_cache_find(_gauge_probe(LATS[2], fields[2], pm), lqcd.F32, 3) is not None
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(10):
        li = int(rng.integers(0, len(LATS)))
        L, bc, th, _ = LATS[li]
        nrhs = int(rng.choice([1, 3]))
        inner = int(rng.choice([lqcd.F64, lqcd.F32]))
        kappa = float(rng.uniform(0.125, 0.136))
        eta = np.stack([inputs.gaussian_spinor(L, 100 + 10 * k + j, bc) for j in range(nrhs)])
        p = lqcd.Server.params(kappa, 1.9, tol=1e-10, inner_prec=inner, nrhs=nrhs)
        reqs.append((li, p, eta))
    # the largest request first, so that later arrivals find it running
    reqs[0] = (2, lqcd.Server.params(0.134, 1.9, tol=1e-10, inner_prec=lqcd.F64, nrhs=6),
               np.stack([inputs.gaussian_spinor(LATS[2][0], 7 + j) for j in range(6)]))
    tickets = []
    for k, (li, p, eta) in enumerate(reqs):
        if k >= 4:
            time.sleep(0.02)
        tickets.append(srv.submit(gids[li], p, eta))
    res = _wait(srv, tickets)
    times = [res[t][2] for t in tickets]  # (submit, admit, done)
    spans = sorted((a, d) for _, a, d in times)
    overlap = any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    # a request submitted while another one was running, and admitted before that one finished
    arrived_during = any(o[1] < s_ < o[2] and a < o[2]
                         for i, (s_, a, _) in enumerate(times) for j, o in enumerate(times) if i != j)
    print(f"served {len(tickets)} requests, overlap={overlap}, arrived_during={arrived_during}, "
          f"peak arena {srv.peak_bytes() / 2**30:.2f} GiB")
    srv.close()
    assert overlap and arrived_during
    # the same solves alone
    for (li, p, eta), t in zip(reqs, tickets):
        st, infos, _, psi = res[t]
        assert st == lqcd.OK, infos
        L, bc, th, _ = LATS[li]
        lat = lqcd.Lattice(L, bc, th)
        g = lqcd.GaugeField(lat, torch.from_numpy(fields[li]), pm)
        alone = lqcd.solve(g, torch.from_numpy(eta).cuda(), p.d.kappa, p.d.csw, tol=p.tol,
                           inner_prec=p.inner_prec).psi.cpu().numpy()
        assert np.array_equal(alone, psi), (li, p.inner_prec, p.nrhs)
    # every column against the oracle
    for (li, p, eta), t in zip(reqs, tickets):
        L, bc, th, _ = LATS[li]
        A = orc.clover_matrix(L, bc, fields[li], orc.m0_from_kappa(p.d.kappa), p.d.csw)
        psi = res[t][3]
        for j in range(p.nrhs):
            r = eta[j] - orc.dw(L, bc, th, fields[li], A, psi[j])
            assert np.linalg.norm(r) / np.linalg.norm(eta[j]) <= 1e-10, (li, j)


def _gauge_probe(lat_spec, U, pm):
    """A gauge-field handle of the same lattice, boundary type and storage as a
    server field (the tuning cache is keyed by those, not by the handle)."""
    L, bc, th, _ = lat_spec
    return lqcd.GaugeField(lqcd.Lattice(L, bc, th), torch.from_numpy(U), pm)


def test_request_with_initial_guess():
    """A request resumed from an earlier result (x0, a host buffer) takes no
    iteration when that result already meets tol, and fewer than from zero
    otherwise; the result meets 1e-10 by the oracle."""
    L, bc, th, sd = LATS[0]
    U = inputs.gauge_field(L, 0.2, seed=sd, bc=bc)
    srv = lqcd.Server(2 << 30, max_streams=2)
    gid = srv.add_gauge(L, bc, th, U, lqcd.PM_F64)
    eta = np.stack([inputs.gaussian_spinor(L, 300 + j, bc) for j in range(2)])
    rough = lqcd.Server.params(0.13, 1.9, tol=1e-6, nrhs=2)
    fine = lqcd.Server.params(0.13, 1.9, tol=1e-10, nrhs=2)
    t0 = srv.submit(gid, rough, eta)
    t1 = srv.submit(gid, fine, eta)
    r0 = _wait(srv, [t0, t1])
    t2 = srv.submit(gid, fine, eta, x0=r0[t0][3])
    # a 1e-10 result resubmitted at 1e-9: its first (FP64) residual meets tol
    t3 = srv.submit(gid, lqcd.Server.params(0.13, 1.9, tol=1e-9, nrhs=2), eta, x0=r0[t1][3])
    r = _wait(srv, [t2, t3])
    srv.close()
    A = orc.clover_matrix(L, bc, U, orc.m0_from_kappa(0.13), 1.9)
    for j in range(2):
        assert r[t2][1][j]["iters"] < r0[t1][1][j]["iters"]
        assert r[t3][1][j]["iters"] == 0
        for t in (t2, t3):
            res = eta[j] - orc.dw(L, bc, th, U, A, r[t][3][j])
            assert r[t][0] == lqcd.OK and np.linalg.norm(res) <= 1e-10 * np.linalg.norm(eta[j])
