"""GPU parity of the direction-split hop kernels (LQCD_TUNE_DIR_SPLIT): two
waves per block of 64 sites, one for the x/y hops and one for the z/t hops,
each producing one chirality of the output.

Same oracle and tolerances as the unsplit kernels (FP64 1e-12 relative, FP32
2e-6, BF16 storage 2e-2; solves: oracle true residual <= 1e-10).  The split
sums the eight hop terms in another order, so it is compared with the oracle,
and bitwise only with itself under the other tuning fields.
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

# 6x4x4x6: V/2 = 288 sites, four full 64-site blocks and a ragged one
CASES = [
    ((6, 4, 4, 6), P, TH_RND, 0.3, 0.1345, 1.9, 1.0),
    ((4, 6, 4, 8), SF, TH_SPATIAL, 0.2, 0.134, 1.8, 1.3),
    ((4, 4, 6, 6), OPEN, TH_SPATIAL, 0.2, 0.13, 1.9, 0.7),
    ((8, 6, 4, 10), P, TH_AP, 0.2, 0.135, 1.9, 1.0),
]
PMASK = {lqcd.F64: lqcd.PM_F64, lqcd.F32: lqcd.PM_F64 | lqcd.PM_F32, lqcd.BF16: lqcd.PM_F64 | lqcd.PM_BF16}


def case_id(c):
    return f"{'x'.join(map(str, c[0]))}-{['P', 'SF', 'OPEN'][c[1]]}"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def g5(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


class Split:
    def __init__(self, L, bc, theta, eps, kappa, csw, cF, seed=17, pm=lqcd.PM_F64):
        self.L, self.bc, self.theta = L, bc, theta
        self.kappa, self.csw, self.cF = kappa, csw, cF
        self.U = inputs.gauge_field(L, eps, seed=seed, bc=bc)
        self.A = orc.clover_matrix(L, bc, self.U, orc.m0_from_kappa(kappa), csw, cF)
        self.lat = lqcd.Lattice(L, bc, theta)
        self.pm = pm
        self.gauge = lqcd.GaugeField(self.lat, torch.from_numpy(self.U), pm)
        self.d = lqcd.dirac(kappa, csw, cF)

    def ws(self, nrhs, prec, **tune):
        w = lqcd.Workspace(self.lat, self.pm & lqcd.PM_PRECISIONS, nrhs)
        cfg = dict(nr_tile=1, block_order=1, rhs_lanes=1, dir_split=True)
        cfg.update(tune)
        lqcd.set_tuning(w, prec, **cfg)
        if prec != lqcd.F64:
            lqcd.set_tuning(w, lqcd.F64, **cfg)
        return w


@pytest.mark.parametrize("prec,tol", [(lqcd.F64, 1e-12), (lqcd.F32, 2e-6), (lqcd.BF16, 2e-2)],
                         ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("c", CASES, ids=case_id)
def test_split_operators_match_oracle(c, prec, tol):
    print(f"\n[gpu case] split {case_id(c)} prec {prec}", flush=True)
    s = Split(*c, pm=PMASK[prec])
    L, bc, th, U, A = s.L, s.bc, s.theta, s.U, s.A
    Ainv = orc.inverse_blocks(A)
    odd = orc.parity_mask(L)
    psi = inputs.gaussian_spinor(L, 5, bc)
    pe = psi.copy()
    pe[odd] = 0
    po = psi.copy()
    po[~odd] = 0
    dh = orc.schur_dhat(L, bc, th, U, A, Ainv, pe)
    dw = orc.dw(L, bc, th, U, A, psi)
    hop_oe = orc.apply_blocks(A, pe) - orc.hop(L, bc, th, U, po)
    hop_oe[odd] = 0
    if bc == SF:
        hop_oe[0] = 0
    refs = ((lqcd.OP_DW, dw), (lqcd.OP_DW_DAG, orc.dw_dag(L, bc, th, U, A, psi)),
            (lqcd.OP_DWDAGDW, orc.dw_dag(L, bc, th, U, A, dw)),
            (lqcd.OP_HOP_EO, orc.schur_hop_eo(L, bc, th, U, Ainv, pe)), (lqcd.OP_HOP_OE, hop_oe),
            (lqcd.OP_SCHUR, dh), (lqcd.OP_SCHUR_DAG, g5(orc.schur_dhat(L, bc, th, U, A, Ainv, g5(pe)))),
            (lqcd.OP_SCHUR_NORMAL, g5(orc.schur_dhat(L, bc, th, U, A, Ainv, g5(dh)))))
    ws = s.ws(1, prec)
    x = torch.from_numpy(np.ascontiguousarray(psi[None])).cuda()
    for op, ref in refs:
        got = lqcd.dw_apply(s.gauge, s.d, x, op=op, prec=prec, ws=ws)
        torch.cuda.synchronize()
        err = rel(got.cpu().numpy()[0], ref)
        print(f"  op {op}: rel err {err:.3e}")
        assert err < tol, (op, err)


def _rho(s, eta, psi):
    r = eta - orc.dw(s.L, s.bc, s.theta, s.U, s.A, psi)
    return float(np.linalg.norm(r) / np.linalg.norm(eta))


@pytest.mark.parametrize("two_row", [False, True], ids=["full", "two_row"])
@pytest.mark.parametrize("c", CASES[:3], ids=case_id)
def test_split_eo_cg_fp64(c, two_row):
    s = Split(*c, seed=23, pm=lqcd.PM_F64 | (lqcd.PM_TWO_ROW if two_row else 0))
    x0 = (0, 0, 0, 1) if s.bc == SF else (0, 0, 0, 0)
    eta = np.stack([inputs.point_source(s.L, x0, 1, 2), inputs.gaussian_spinor(s.L, 9, s.bc)])
    for j in range(2):  # one rhs at a time: the shape the split serves
        r = lqcd.solve(s.gauge, torch.from_numpy(eta[j:j + 1]).cuda(), s.kappa, s.csw, s.cF, tol=1e-10,
                       ws=s.ws(1, lqcd.F64), use_graph=True, stream=torch.cuda.Stream())
        torch.cuda.synchronize()
        rho = _rho(s, eta[j], r.psi.cpu().numpy()[0])
        print(f"split {case_id(c)} two_row={two_row} rhs {j}: iters {r.info[0]['iters']} rho {rho:.3e}")
        assert r.status == lqcd.OK and rho <= 1e-10


@pytest.mark.parametrize("inner", [lqcd.F32, lqcd.BF16], ids=["f32", "bf16"])
def test_split_mixed_precision(inner):
    s = Split((8, 8, 8, 16), P, TH_AP, 0.2, 0.135, 1.9, 1.0, seed=3, pm=PMASK[inner])
    eta = inputs.z2_noise(s.L, seed=3)
    r = lqcd.solve(s.gauge, torch.from_numpy(eta[None]).cuda(), s.kappa, s.csw, tol=1e-10, inner_prec=inner,
                   reliable_every=100, maxiter=20000, ws=s.ws(1, inner))
    rho = _rho(s, eta, r.psi.cpu().numpy()[0])
    print(f"split mixed {inner}: iters {r.info[0]['iters']} rho {rho:.3e}")
    assert r.status == lqcd.OK and rho <= 1e-10


def test_split_is_bitwise_stable_under_the_other_tuning_fields():
    """With the split on, block order, store and load kinds and occupancy caps
    leave the solution bitwise unchanged (graph-captured and eager alike)."""
    s = Split((16, 16, 8, 8), P, TH_AP, 0.2, 0.134, 1.9, 1.0, seed=8,
              pm=lqcd.PM_F64 | lqcd.PM_BF16)
    eta = torch.from_numpy(inputs.gaussian_spinor(s.L, 4)[None]).cuda()
    for ip in (lqcd.F64, lqcd.BF16):
        ref = None
        for order, nt, cached, occ, graph in ((0, False, False, 0, False), (2, True, True, 1, True),
                                               (5, True, False, 3, True), (6, False, True, 2, False)):
            ws = s.ws(1, ip, block_order=order, nt_store=nt, cached_gauge=cached, occ_cap=occ)
            r = lqcd.solve(s.gauge, eta, s.kappa, s.csw, tol=1e-10, inner_prec=ip, ws=ws, use_graph=graph,
                           stream=torch.cuda.Stream())
            torch.cuda.synchronize()
            got = r.psi.cpu().numpy()
            if ref is None:
                ref = got
                assert _rho(s, inputs.gaussian_spinor(s.L, 4), got[0]) <= 1e-10
            assert np.array_equal(got, ref), (ip, order, nt, cached, occ)


def test_autotune_keeps_the_split_setting():
    s = Split((8, 8, 8, 16), P, TH_AP, 0.2, 0.135, 1.9, 1.0, seed=9)
    for split in (True, False):
        ws = s.ws(1, lqcd.F64, dir_split=split)
        best, us = lqcd.autotune(s.gauge, s.d, lqcd.F64, 1, ws)
        assert best["dir_split"] == split and lqcd.get_tuning(ws, lqcd.F64)["dir_split"] == split and us > 0
