"""Parity at the full workload sizes, in the launch configuration the
benchmark times (two-row links; the benchmark step's tuning with the
direction split at 16^3x32, autotuned hop kernels with the split for one rhs
elsewhere; graph-captured chunks): the 16^3x32 step lattice (kappa 0.1345,
csw 1.9), the 32^3x64 periodic/antiperiodic lattice (kappa 0.135, csw 1.9)
and the 24^3x48 Schroedinger-functional lattice (kappa 0.134, csw 1.8),
checked against the oracle on the whole lattice (its Dw is cheap enough
here)."""
import numpy as np
import pytest
import torch

import bench
from oracle import oracle as orc
from paper_2503_16994_amd import inputs, lqcd

pytestmark = pytest.mark.gpu

PM = lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_BF16
GPM = PM | lqcd.PM_TWO_ROW  # gauge fields, as in the benchmark


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c2_step_configuration_16x16x16x32():
    """The benchmark step exactly: two-row links, the step's tuning (direction
    split), graph chunks on a side stream, the 12 point sources solved one at
    a time; every solution checked with the oracle operator; and the
    roofline kernel (the o->e hop in that tuning) against the oracle."""
    L, kappa, csw = bench.L_C2, bench.KAPPA, bench.CSW
    U = inputs.gauge_field(L, bench.EPS, seed=bench.SEED)
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, bench.THETA)
    g = lqcd.GaugeField(lat, torch.from_numpy(U), lqcd.PM_F64 | lqcd.PM_TWO_ROW)
    A = orc.clover_matrix(L, orc.PERIODIC, U, orc.m0_from_kappa(kappa), csw)
    ws = lqcd.Workspace(lat, lqcd.PM_F64, 1)
    lqcd.set_tuning(ws, lqcd.F64, *bench.STEP_TUNING)
    eta = torch.from_numpy(inputs.point_sources_12(L)).cuda()
    psi = torch.empty_like(eta)
    stream = torch.cuda.Stream()
    infos = [lqcd.solve(g, eta[j:j + 1], kappa, csw, tol=bench.TOL, inner_prec=lqcd.F64, use_graph=True, ws=ws,
                        stream=stream, psi=psi[j:j + 1]).info[0] for j in range(12)]
    torch.cuda.synchronize()
    e, p = eta.cpu().numpy(), psi.cpu().numpy()
    for j in range(12):
        r = e[j] - orc.dw(L, orc.PERIODIC, bench.THETA, U, A, p[j])
        rho = float(np.linalg.norm(r) / np.linalg.norm(e[j]))
        assert infos[j]["status"] == 0 and rho <= 1e-10, (j, rho)
    # the roofline kernel: HOP_OE = A_ee x_e - D_eo y_o on the even sites
    d = lqcd.dirac(kappa, csw)
    x = inputs.gaussian_spinor(L, 12)
    odd = orc.parity_mask(L)
    xe, yo = x.copy(), x.copy()
    xe[odd] = 0
    yo[~odd] = 0
    ref = orc.apply_blocks(A, xe) - orc.hop(L, orc.PERIODIC, bench.THETA, U, yo)
    ref[odd] = 0
    got = lqcd.dw_apply(g, d, torch.from_numpy(x[None]).cuda(), op=lqcd.OP_HOP_OE, prec=lqcd.F64, ws=ws)
    torch.cuda.synchronize()
    assert rel(got.cpu().numpy()[0], ref) < 1e-12


@pytest.fixture(scope="module")
def c3():
    L, kappa, csw, th = (32, 32, 32, 64), 0.135, 1.9, (1, 1, 1, -1)
    U = inputs.gauge_field(L, 0.2, seed=3)
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, th)
    g = lqcd.GaugeField(lat, torch.from_numpy(U), GPM)
    A = orc.clover_matrix(L, orc.PERIODIC, U, orc.m0_from_kappa(kappa), csw)
    yield dict(L=L, kappa=kappa, csw=csw, th=th, U=U, A=A, lat=lat, g=g)
    del g
    torch.cuda.empty_cache()


def test_operator_32x32x32x64_fp64_matches_oracle(c3):
    ws = lqcd.Workspace(c3["lat"], PM, 1)
    d = lqcd.dirac(c3["kappa"], c3["csw"])
    lqcd.set_tuning(ws, lqcd.F64, dir_split=True)
    best, _ = lqcd.autotune(c3["g"], d, lqcd.F64, 1, ws)
    psi = inputs.gaussian_spinor(c3["L"], 11)
    got = lqcd.dw_apply(c3["g"], d, torch.from_numpy(psi[None]).cuda(), lqcd.OP_DW, lqcd.F64, ws).cpu().numpy()[0]
    ref = orc.dw(c3["L"], orc.PERIODIC, c3["th"], c3["U"], c3["A"], psi)
    err = rel(got, ref)
    print(f"32^3x64 FP64 Dw, tuning {best}: rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("inner", [lqcd.F32, lqcd.BF16], ids=["f32", "bf16"])
def test_mixed_solve_32x32x32x64_z2_source(c3, inner):
    ws = lqcd.Workspace(c3["lat"], PM, 1)
    d = lqcd.dirac(c3["kappa"], c3["csw"])
    lqcd.set_tuning(ws, inner, dir_split=True)
    lqcd.autotune(c3["g"], d, inner, 1, ws)
    eta = inputs.z2_noise(c3["L"], seed=3)
    stream = torch.cuda.Stream()
    r = lqcd.solve(c3["g"], torch.from_numpy(eta[None]).cuda(), c3["kappa"], c3["csw"], tol=1e-10,
                   inner_prec=inner, reliable_every=100, use_graph=True, ws=ws, stream=stream)
    torch.cuda.synchronize()
    psi = r.psi.cpu().numpy()[0]
    res = eta - orc.dw(c3["L"], orc.PERIODIC, c3["th"], c3["U"], c3["A"], psi)
    rho = float(np.linalg.norm(res) / np.linalg.norm(eta))
    print(f"32^3x64 Z2 inner {inner}: iters {r.info[0]['iters']} rho(oracle) {rho:.3e} "
          f"rho(gpu) {r.info[0]['true_residual']:.3e}")
    assert r.status == lqcd.OK and rho <= 1e-10


@pytest.fixture(scope="module")
def c4():
    L, kappa, csw, th = (24, 24, 24, 48), 0.134, 1.8, (1, 1, 1, 1)
    U = inputs.gauge_field(L, 0.2, seed=4, bc=orc.SF)
    lat = lqcd.Lattice(L, lqcd.BC_SF, th)
    g = lqcd.GaugeField(lat, torch.from_numpy(U), GPM)
    A = orc.clover_matrix(L, orc.SF, U, orc.m0_from_kappa(kappa), csw)
    yield dict(L=L, kappa=kappa, csw=csw, th=th, U=U, A=A, lat=lat, g=g)
    del g
    torch.cuda.empty_cache()


@pytest.mark.parametrize("inner", [lqcd.F64, lqcd.F32, lqcd.BF16], ids=["f64", "f32", "bf16"])
def test_multi_rhs_24x24x24x48_sf_twelve_sources(c4, inner):
    """The 24^3x48 SF workload: the 12 point sources at t = 1 in one 12-rhs
    solve, FP64, FP32 or BF16 inner precision with FP64 reliable updates
    every 100 iterations, autotuned kernels, graph chunks, and the FP64 hops
    of the reliable updates with the direction split (the benchmark's mixed
    legs); every column's residual recomputed by the oracle <= 1e-10."""
    L, kappa, csw, th = c4["L"], c4["kappa"], c4["csw"], c4["th"]
    print(f"\n[gpu case] 24^3x48 SF 12 rhs inner {inner}", flush=True)
    ws = lqcd.Workspace(c4["lat"], PM, 12)
    d = lqcd.dirac(kappa, csw)
    best, _ = lqcd.autotune(c4["g"], d, inner, 12, ws)
    if inner != lqcd.F64:
        t64 = lqcd.get_tuning(ws, lqcd.F64)
        t64["dir_split"] = True
        lqcd.set_tuning(ws, lqcd.F64, **t64)
    eta = inputs.point_sources_12(L, (0, 0, 0, 1))
    stream = torch.cuda.Stream()
    r = lqcd.solve(c4["g"], torch.from_numpy(eta).cuda(), kappa, csw, tol=1e-10, inner_prec=inner,
                   reliable_every=100, use_graph=True, ws=ws, stream=stream)
    torch.cuda.synchronize()
    psi = r.psi.cpu().numpy()
    worst = 0.0
    for j in range(12):
        res = eta[j] - orc.dw(L, orc.SF, th, c4["U"], c4["A"], psi[j])
        worst = max(worst, float(np.linalg.norm(res) / np.linalg.norm(eta[j])))
        assert np.all(psi[j, 0] == 0)  # Dirichlet slice
    print(f"24^3x48 SF 12 rhs inner {inner}, tuning {best}: max iters "
          f"{max(i['iters'] for i in r.info)}, fp64 from {[i['fp64_from'] for i in r.info]}, "
          f"max rho(oracle) {worst:.3e}")
    assert r.status == lqcd.OK and worst <= 1e-10
    del ws
    torch.cuda.empty_cache()
