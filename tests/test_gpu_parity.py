"""GPU parity: the gfx950 library against the FP64 oracle, through the C ABI.

Tolerances:
* FP64 operator applications: relative 2-norm difference <= 1e-12 (the two
  sides sum the same terms in different orders; the observed difference is
  ~1e-16).
* FP32 storage/arithmetic: <= 2e-6 relative (a few units of 2^-24 times the
  ~20 terms per output component).
* BF16 storage (links, clover, spinors) with FP32 arithmetic: <= 2e-2
  (several inputs each rounded to 2^-9 relative, plus the rounded output).
* Solves: the true residual |eta - Dw psi| / |eta| recomputed by the oracle
  must be <= tol (1e-12 for the 4^4 full-lattice case, 1e-10 otherwise); the
  error against the oracle's own solution is reported and bounded by
  cond(Dw) * (rho_gpu + rho_oracle).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_16994_amd import inputs, lqcd

pytestmark = pytest.mark.gpu

P, SF, OPEN = 0, 1, 2
TH_AP = (1, 1, 1, -1)
TH_RND = tuple(np.exp(1j * np.array([0.3, -1.2, 2.2, 0.7])))
TH_SPATIAL = tuple(np.exp(1j * np.array([0.3, -1.2, 2.2, 0.0])))

# (L, bc, theta, eps, kappa, csw, cF); the 6x4x4x6 lattice has V/2 = 288 sites,
# i.e. two full 128-thread workgroups and a ragged one (and a ragged 64-site
# layout tile).
OP_CASES = [
    ((4, 4, 4, 4), P, TH_AP, 0.3, 0.12, 1.0, 1.0),
    ((6, 4, 4, 6), P, TH_RND, 0.3, 0.1345, 1.9, 1.0),
    ((4, 6, 4, 8), SF, TH_SPATIAL, 0.2, 0.134, 1.8, 1.3),
    ((4, 4, 6, 6), OPEN, TH_SPATIAL, 0.2, 0.13, 1.9, 0.7),
    ((8, 6, 4, 10), P, TH_AP, 0.2, 0.135, 1.9, 1.0),
]


def case_id(c):
    L, bc, *_ = c
    return f"{'x'.join(map(str, L))}-{['P', 'SF', 'OPEN'][bc]}"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def g5(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


class Setup:
    def __init__(self, L, bc, theta, eps, kappa, csw, cF, seed=17, pmask=lqcd.PM_F64):
        self.L, self.bc, self.theta = L, bc, theta
        self.kappa, self.csw, self.cF = kappa, csw, cF
        self.m0 = orc.m0_from_kappa(kappa)
        self.U = inputs.gauge_field(L, eps, seed=seed, bc=bc)
        self.A = orc.clover_matrix(L, bc, self.U, self.m0, csw, cF)
        self.lat = lqcd.Lattice(L, bc, theta)
        self.gauge = lqcd.GaugeField(self.lat, torch.from_numpy(self.U), pmask)
        self.d = lqcd.dirac(kappa, csw, cF)

    def fields(self, n, seed=0):
        return np.stack([inputs.gaussian_spinor(self.L, seed + i, self.bc) for i in range(n)])

    def apply(self, psi, op, prec=lqcd.F64, ws=None):
        x = torch.from_numpy(np.ascontiguousarray(psi)).cuda()
        out = lqcd.dw_apply(self.gauge, self.d, x, op=op, prec=prec, ws=ws)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    # oracle side
    def o_dw(self, psi):
        return orc.dw(self.L, self.bc, self.theta, self.U, self.A, psi)

    def o_dwdag(self, psi):
        return orc.dw_dag(self.L, self.bc, self.theta, self.U, self.A, psi)


@pytest.fixture(scope="module", params=OP_CASES, ids=case_id)
def setup(request):
    print(f"\n[gpu case] {case_id(request.param)}", flush=True)
    return Setup(*request.param)


def test_full_operator_fp64(setup):
    s = setup
    psi = s.fields(2, seed=3)
    ws = lqcd.Workspace(s.lat, lqcd.PM_F64, 2)
    expect = {
        lqcd.OP_DW: [s.o_dw(p) for p in psi],
        lqcd.OP_DW_DAG: [s.o_dwdag(p) for p in psi],
        lqcd.OP_G5DW: [g5(s.o_dw(p)) for p in psi],
        lqcd.OP_DWDAGDW: [s.o_dwdag(s.o_dw(p)) for p in psi],
    }
    for op, exp in expect.items():
        got = s.apply(psi, op, ws=ws)
        for j in range(2):
            assert rel(got[j], exp[j]) < 1e-12, (op, j, rel(got[j], exp[j]))


def test_schur_operators_fp64(setup):
    s = setup
    L, bc, th = s.L, s.bc, s.theta
    Ainv = orc.inverse_blocks(s.A)
    odd = orc.parity_mask(L)
    psi = s.fields(1, seed=11)[0]
    pe = psi.copy()
    pe[odd] = 0
    po = psi.copy()
    po[~odd] = 0

    def dhat(v):
        return orc.schur_dhat(L, bc, th, s.U, s.A, Ainv, v)

    got = s.apply(psi[None], lqcd.OP_SCHUR)[0]
    assert rel(got, dhat(pe)) < 1e-12
    got = s.apply(psi[None], lqcd.OP_SCHUR_DAG)[0]
    assert rel(got, g5(dhat(g5(pe)))) < 1e-12
    got = s.apply(psi[None], lqcd.OP_SCHUR_NORMAL)[0]
    assert rel(got, g5(dhat(g5(dhat(pe))))) < 1e-12
    got = s.apply(psi[None], lqcd.OP_HOP_EO)[0]
    assert rel(got, orc.schur_hop_eo(L, bc, th, s.U, Ainv, pe)) < 1e-12
    # HOP_OE: A_ee x_e - D_eo y_o on the even sites
    exp = orc.apply_blocks(s.A, pe) - orc.hop(L, bc, th, s.U, po)
    exp[odd] = 0
    if bc == SF:
        exp[0] = 0
    got = s.apply(psi[None], lqcd.OP_HOP_OE)[0]
    assert rel(got, exp) < 1e-12
    # the clover blocks alone: HOP_OE with a zero odd part is A_ee on the even sites
    clov = orc.apply_blocks(s.A, pe)
    if bc == SF:
        clov[0] = 0
    got = s.apply(pe[None], lqcd.OP_HOP_OE)[0]
    assert rel(got, clov) < 1e-12


@pytest.mark.parametrize("prec,tol", [(lqcd.F32, 2e-6), (lqcd.BF16, 2e-2)], ids=["f32", "bf16"])
@pytest.mark.parametrize("c", OP_CASES[1:4], ids=case_id)
def test_reduced_precision_operator(c, prec, tol):
    pm = lqcd.PM_F64 | (lqcd.PM_F32 if prec == lqcd.F32 else lqcd.PM_BF16)
    s = Setup(*c, pmask=pm)
    psi = s.fields(1, seed=5)
    ws = lqcd.Workspace(s.lat, pm, 1)
    Ainv = orc.inverse_blocks(s.A)
    odd = orc.parity_mask(s.L)
    pe = psi[0].copy()
    pe[odd] = 0
    dh = orc.schur_dhat(s.L, s.bc, s.theta, s.U, s.A, Ainv, pe)
    cases = ((lqcd.OP_DW, s.o_dw(psi[0])), (lqcd.OP_DWDAGDW, s.o_dwdag(s.o_dw(psi[0]))),
             (lqcd.OP_HOP_EO, orc.schur_hop_eo(s.L, s.bc, s.theta, s.U, Ainv, pe)),
             (lqcd.OP_SCHUR, dh),
             (lqcd.OP_SCHUR_NORMAL, g5(orc.schur_dhat(s.L, s.bc, s.theta, s.U, s.A, Ainv, g5(dh)))))
    for op, ref in cases:
        got = s.apply(psi, op, prec=prec, ws=ws)[0]
        err = rel(got, ref)
        print(f"{case_id(c)} prec {prec} op {op}: rel err {err:.3e}")
        assert err < tol


def _oracle_rho(s, eta, psi):
    r = eta - s.o_dw(psi)
    return float(np.linalg.norm(r) / np.linalg.norm(eta))


def test_c1_full_cg_4x4x4x4():
    """Plain FP64 full-lattice CG on Dw^+ Dw, 4^4, point source, 1e-12."""
    s = Setup((4, 4, 4, 4), P, TH_AP, 0.3, 0.12, 1.0, 1.0, seed=1)
    eta = inputs.point_source(s.L, (0, 0, 0, 0), 0, 0)
    res = lqcd.solve(s.gauge, torch.from_numpy(eta).cuda(), s.kappa, s.csw, tol=1e-12,
                     solver=lqcd.SOLVER_CG_FULL)
    psi = res.psi.cpu().numpy()
    rho = _oracle_rho(s, eta, psi)
    ref, rho_o, it_o, ok = orc.cg(s.L, P, TH_AP, s.U, s.A, eta, tol=1e-12)
    print(f"C1: gpu iters {res.info[0]['iters']} rho {rho:.3e}; oracle iters {it_o} rho {rho_o:.3e}; "
          f"|psi-psi_or|/|psi_or| = {rel(psi, ref):.3e}")
    assert res.status == lqcd.OK
    assert rho <= 1e-12 and abs(rho - res.info[0]["true_residual"]) < 1e-14
    assert rel(psi, ref) < 1e-9


@pytest.mark.parametrize("c", OP_CASES[:4], ids=case_id)
def test_eo_cg_fp64_every_boundary(c):
    s = Setup(*c, seed=23)
    x0 = (0, 0, 0, 1) if s.bc == SF else (0, 0, 0, 0)
    eta = np.stack([inputs.point_source(s.L, x0, 1, 2), inputs.gaussian_spinor(s.L, 9, s.bc)])
    res = lqcd.solve(s.gauge, torch.from_numpy(eta).cuda(), s.kappa, s.csw, s.cF, tol=1e-10)
    psi = res.psi.cpu().numpy()
    for j in range(2):
        rho = _oracle_rho(s, eta[j], psi[j])
        ref, rho_o, _, ok = orc.cg(s.L, s.bc, s.theta, s.U, s.A, eta[j], tol=1e-10)
        print(f"{case_id(c)} rhs {j}: iters {res.info[j]['iters']} rho {rho:.3e} err {rel(psi[j], ref):.3e}")
        assert rho <= 1e-10
        assert rel(psi[j], ref) < 1e-7
    if s.bc == SF:
        assert np.all(psi[:, 0] == 0)


def test_c2_eo_cg_fp64_16x16x16x32_twelve_sources():
    """Plain FP64 even-odd CG, 16^3x32, 12 point sources solved one at a time."""
    s = Setup((16, 16, 16, 32), P, TH_AP, 0.2, 0.1345, 1.9, 1.0, seed=2)
    ws = lqcd.Workspace(s.lat, lqcd.PM_F64, 1)
    for j in range(12):
        eta = inputs.point_source(s.L, (0, 0, 0, 0), j // 3, j % 3)
        res = lqcd.solve(s.gauge, torch.from_numpy(eta).cuda(), s.kappa, s.csw, tol=1e-10, ws=ws)
        psi = res.psi.cpu().numpy()
        rho = _oracle_rho(s, eta, psi)
        print(f"C2 source {j}: iters {res.info[0]['iters']} restarts {res.info[0]['restarts']} "
              f"rho(oracle) {rho:.3e} rho(gpu) {res.info[0]['true_residual']:.3e} "
              f"t {res.info[0]['seconds']:.3f}s", flush=True)
        assert res.status == lqcd.OK
        assert rho <= 1e-10


@pytest.mark.parametrize("inner", [lqcd.F32, lqcd.BF16], ids=["f32", "bf16"])
def test_mixed_precision_eo_cg(inner):
    pm = lqcd.PM_F64 | (lqcd.PM_F32 if inner == lqcd.F32 else lqcd.PM_BF16)
    s = Setup((8, 8, 8, 16), P, TH_AP, 0.2, 0.135, 1.9, 1.0, seed=3, pmask=pm)
    eta = inputs.z2_noise(s.L, seed=3)
    res = lqcd.solve(s.gauge, torch.from_numpy(eta).cuda(), s.kappa, s.csw, tol=1e-10,
                     inner_prec=inner, reliable_every=100, maxiter=20000)
    psi = res.psi.cpu().numpy()
    rho = _oracle_rho(s, eta, psi)
    ref, rho_o, it_o, _ = orc.cg(s.L, P, TH_AP, s.U, s.A, eta, tol=1e-10)
    print(f"mixed {inner}: iters {res.info[0]['iters']} reliable updates {res.info[0]['reliable_updates']} "
          f"rho {rho:.3e} err vs oracle {rel(psi, ref):.3e} (oracle iters {it_o})")
    assert res.status == lqcd.OK
    assert rho <= 1e-10


def test_multi_rhs_equals_single_rhs_bitwise():
    s = Setup((8, 8, 8, 8), P, TH_AP, 0.2, 0.134, 1.9, 1.0, seed=4)
    eta = inputs.point_sources_12(s.L, (0, 0, 0, 0))[:6] + 0.1 * np.stack(
        [inputs.gaussian_spinor(s.L, k) for k in range(6)])
    e = torch.from_numpy(eta).cuda()
    batch = lqcd.solve(s.gauge, e, s.kappa, s.csw, tol=1e-10).psi.cpu().numpy()
    for j in range(6):
        alone = lqcd.solve(s.gauge, e[j:j + 1], s.kappa, s.csw, tol=1e-10).psi.cpu().numpy()[0]
        assert np.array_equal(alone, batch[j]), j


def test_graph_capture_matches_eager_and_is_deterministic():
    s = Setup((8, 8, 8, 8), P, TH_AP, 0.2, 0.134, 1.9, 1.0, seed=6)
    eta = torch.from_numpy(inputs.z2_noise(s.L, 1)[None]).cuda()
    stream = torch.cuda.Stream()
    eager = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=1e-10, stream=stream).psi.cpu().numpy()
    for _ in range(3):
        g = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=1e-10, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        assert np.array_equal(g.psi.cpu().numpy(), eager)


def test_graph_chunks_of_both_lengths_match_eager(capfd, monkeypatch):
    """Near convergence the solver switches from 50- to 10-iteration chunks
    (a second cached graph; predicted from the |r|^2 decay between polls, so
    only solves longer than 100 iterations can use it); the chunking never
    changes a result: graph-captured 12-rhs BF16-inner solves on 16^3x32
    (replayed three times, eager work in between) equal the eager solve bit
    for bit, with equal iteration counts, and at tol 1e-10 (105 iterations)
    the last chunk is a short one."""
    s = Setup((16, 16, 16, 32), P, TH_AP, 0.2, 0.1345, 1.9, 1.0, seed=2,
              pmask=lqcd.PM_F64 | lqcd.PM_BF16)
    eta = torch.from_numpy(inputs.point_sources_12(s.L, (0, 0, 0, 0))).cuda()
    stream = torch.cuda.Stream()
    monkeypatch.setenv("LQCD_TRACE", "1")
    seen = []
    for tol in (1e-10, 1e-9):
        ws = lqcd.Workspace(s.lat, s.gauge.pmask, 12)
        eager = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=tol, inner_prec=lqcd.BF16, ws=ws, stream=stream)
        torch.cuda.synchronize()
        ref, iters = eager.psi.cpu().numpy(), [i["iters"] for i in eager.info]
        for _ in range(3):
            g = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=tol, inner_prec=lqcd.BF16, ws=ws, stream=stream,
                           use_graph=True)
            torch.cuda.synchronize()
            assert g.status == lqcd.OK and [i["iters"] for i in g.info] == iters, tol
            assert np.array_equal(g.psi.cpu().numpy(), ref), tol
            lqcd.dw_apply(s.gauge, lqcd.dirac(s.kappa, s.csw), eta[:1], stream=stream)  # eager work between
        seen.append((tol, max(iters), capfd.readouterr().err.count("next chunk 10")))
    assert any(n > 0 for _, it, n in seen if it > 100), seen


def test_tuning_does_not_change_results():
    """rhs tile, block order, rhs lanes, store and load kinds and occupancy caps
    leave every rhs bitwise equal."""
    # 16x16x8x8: Lz % 8 == 0 and (Lx/2) Ly = 128, so block orders 2 and 5 are
    # exercised (6 needs Lz % 16 == 0 and falls back to 1 here)
    s = Setup((16, 16, 8, 8), P, TH_AP, 0.2, 0.134, 1.9, 1.0, seed=8,
              pmask=lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_BF16)
    eta = torch.from_numpy(np.stack([inputs.gaussian_spinor(s.L, k) for k in range(8)])).cuda()
    ref = {}
    for ip in (lqcd.F64, lqcd.F32, lqcd.BF16):
        for cfg in ((1, 0, 1, False, False, 0), (2, 1, 1, True, True, 1), (3, 2, 2, False, True, 3),
                    (1, 3, 2, True, False, 2), (1, 4, 4, False, False, 0), (2, 5, 4, True, True, 3),
                    (3, 6, 1, True, False, 0)):
            ws = lqcd.Workspace(s.lat, s.gauge.pmask, 8)
            lqcd.set_tuning(ws, ip, *cfg)
            assert lqcd.get_tuning(ws, ip)["nr_tile"] == cfg[0]
            if ip == lqcd.F64 and cfg[2] > 1:
                continue
            r = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=1e-10, inner_prec=ip, ws=ws)
            got = r.psi.cpu().numpy()
            if ip not in ref:
                ref[ip] = got
            assert np.array_equal(got, ref[ip]), (ip, cfg)


def test_autotune_picks_a_valid_config():
    s = Setup((8, 8, 8, 16), P, TH_AP, 0.2, 0.135, 1.9, 1.0, seed=9, pmask=lqcd.PM_F64 | lqcd.PM_F32)
    ws = lqcd.Workspace(s.lat, s.gauge.pmask, 12)
    best, us = lqcd.autotune(s.gauge, s.d, lqcd.F32, 12, ws)
    print("autotune 8^3x16 F32 N=12:", best, f"{us:.1f} us")
    assert best["nr_tile"] in (1, 2, 3) and us > 0
    assert lqcd.get_tuning(ws, lqcd.F32) == best
    eta = torch.from_numpy(inputs.point_sources_12(s.L)).cuda()
    r = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=1e-10, inner_prec=lqcd.F32, ws=ws)
    assert r.status == lqcd.OK


def test_mixed_precision_stall_continues_in_fp64():
    """BF16 inner precision on a Schroedinger-functional system whose
    conditioning it cannot resolve (without the continuation it stagnates at
    a true residual ~1e-7): the stalled rhs must continue in FP64 and still
    reach the tolerance, checked with the oracle operator."""
    L = (8, 8, 8, 32)
    s = Setup(L, SF, (1, 1, 1, 1), 0.2, 0.134, 1.8, 1.0, seed=4,
              pmask=lqcd.PM_F64 | lqcd.PM_BF16)
    eta = np.stack([inputs.point_source(L, (0, 0, 0, 1), 0, 0), inputs.point_source(L, (0, 0, 0, 1), 3, 2)])
    res = lqcd.solve(s.gauge, torch.from_numpy(eta).cuda(), s.kappa, s.csw, tol=1e-10,
                     inner_prec=lqcd.BF16, maxiter=20000)
    psi = res.psi.cpu().numpy()
    for j in range(2):
        rho = _oracle_rho(s, eta[j], psi[j])
        print(f"SF bf16 rhs {j}: iters {res.info[j]['iters']} fp64 from {res.info[j]['fp64_from']} "
              f"rho {rho:.3e}")
        assert rho <= 1e-10
        assert res.info[j]["fp64_from"] > 0
    assert res.status == lqcd.OK


@pytest.mark.parametrize("inner", [lqcd.F64, lqcd.F32], ids=["f64", "f32"])
def test_zero_source_column(inner):
    """A batch whose second column is identically zero: that column is done at
    setup with psi = 0 exactly, the others converge as usual."""
    pm = lqcd.PM_F64 | lqcd.PM_F32
    s = Setup((6, 4, 4, 6), P, TH_RND, 0.3, 0.1345, 1.9, 1.0, seed=12, pmask=pm)
    eta = np.stack([inputs.gaussian_spinor(s.L, 1), np.zeros(s.lat.spinor_shape(), np.complex128),
                    inputs.point_source(s.L, (1, 2, 3, 4), 2, 1)])
    res = lqcd.solve(s.gauge, torch.from_numpy(eta).cuda(), s.kappa, s.csw, tol=1e-10, inner_prec=inner)
    psi = res.psi.cpu().numpy()
    assert res.status == lqcd.OK
    assert np.all(psi[1] == 0) and res.info[1]["iters"] == 0 and res.info[1]["true_residual"] == 0.0
    for j in (0, 2):
        assert _oracle_rho(s, eta[j], psi[j]) <= 1e-10
