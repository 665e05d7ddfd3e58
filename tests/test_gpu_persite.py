"""Per-site parity of the FP32 and BF16 hop kernels against the oracle fed
the same rounded operands.

The GPU stores links, clover blocks and input spinors in FP32 or BF16
(round-to-nearest-even from FP64, BF16 through FP32) and computes in FP32.
Here the test rounds the oracle's own links, clover blocks (A on the even
sites, A^{-1} on the odd sites, per 6x6 chirality block) and input the same
way with numpy, and the oracle applies the hop launch in FP64 to those
rounded operands.  What is left between the two results is the GPU's FP32
arithmetic and the rounding of its output, so every component of every site
must satisfy

    |gpu - ref| <= u_out |ref| + 64 * 2^-24 * S(x),

with u_out the unit roundoff of the output (2^-8 BF16, 2^-24 FP32: the
output rounding alone) and S(x) the site's magnitude scale: the Frobenius
norm of its clover block times the sum over the eight hops of |U|_F |psi|,
plus |A|_F |z| for the self term (a bound on the size of the terms whose
FP32 sum the kernel forms; 64 roundings cover the longest chain of the
sum).  A wrong hop, phase, projector, link or block at one site makes an
error of the size of its terms there, which is far outside this bound.
Rounding the clover blocks of the oracle rather than the GPU's own is exact
except where an FP64 difference in the last bit straddles a rounding
boundary, which does not happen at these sizes.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_16994_amd import inputs, lqcd

pytestmark = pytest.mark.gpu

P, SF, OPEN = 0, 1, 2
TH_RND = tuple(np.exp(1j * np.array([0.3, -1.2, 2.2, 0.7])))
TH_SPATIAL = tuple(np.exp(1j * np.array([0.3, -1.2, 2.2, 0.0])))
CASES = [
    ((6, 4, 4, 6), P, TH_RND, 0.3, 0.1345, 1.9, 1.0),
    ((4, 6, 4, 8), SF, TH_SPATIAL, 0.2, 0.134, 1.8, 1.3),
    ((4, 4, 6, 6), OPEN, TH_SPATIAL, 0.2, 0.13, 1.9, 0.7),
]
# (name, nrhs, tuning kwargs): one rhs per thread, the direction split,
# three rhs per thread (the look-ahead BF16 path and the plain FP32 path of
# the multi-rhs kernels), two lanes per site
TUNINGS = [
    ("nr1", 1, {}),
    ("split", 1, {"dir_split": True}),
    ("nr3", 3, {"nr_tile": 3}),
    ("lanes2", 2, {"rhs_lanes": 2}),
]


def case_id(c):
    L, bc, *_ = c
    return f"{'x'.join(map(str, L))}-{['P', 'SF', 'OPEN'][bc]}"


def round_f32(x):
    x = np.asarray(x, np.complex128)
    return x.real.astype(np.float32).astype(np.float64) + 1j * x.imag.astype(np.float32).astype(np.float64)


def _bf16(a):
    f = np.ascontiguousarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16  # round to nearest even on the 16 dropped bits
    return (u.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def round_bf16(x):
    x = np.asarray(x, np.complex128)
    return _bf16(x.real) + 1j * _bf16(x.imag)


def test_bf16_rounding_emulation():
    """The numpy emulation rounds to nearest even: exact halves go to the
    even neighbour, everything else to the nearest BF16 value."""
    one = 1.0
    ulp = 2.0 ** -7  # BF16 spacing in [1, 2)
    cases = [(one + 0.5 * ulp, one), (one + 1.5 * ulp, one + 2 * ulp), (one + 0.49 * ulp, one),
             (one + 0.51 * ulp, one + ulp), (-(one + 0.51 * ulp), -(one + ulp)), (3.0, 3.0)]
    for v, e in cases:
        assert _bf16(np.array([v]))[0] == e, (v, e)


def _blocks_rounded(M, rnd):
    """Round the two 6x6 chirality blocks of 12x12 site matrices (the
    off-block zeros stay exact zeros, the diagonal is real)."""
    out = rnd(M)
    return out


class Case:
    def __init__(self, L, bc, theta, eps, kappa, csw, cF, prec):
        self.L, self.bc, self.theta, self.prec = L, bc, theta, prec
        self.U = inputs.gauge_field(L, eps, seed=41, bc=bc)
        self.A = orc.clover_matrix(L, bc, self.U, orc.m0_from_kappa(kappa), csw, cF)
        self.Ainv = orc.inverse_blocks(self.A)
        pm = lqcd.PM_F64 | (lqcd.PM_F32 if prec == lqcd.F32 else lqcd.PM_BF16)
        self.lat = lqcd.Lattice(L, bc, theta)
        self.gauge = lqcd.GaugeField(self.lat, torch.from_numpy(self.U), pm)
        self.d = lqcd.dirac(kappa, csw, cF)
        self.pm = pm
        self.rnd = round_f32 if prec == lqcd.F32 else round_bf16
        self.u_out = 2.0 ** -24 if prec == lqcd.F32 else 2.0 ** -8
        Ur = self.rnd(self.U)
        if bc == OPEN:  # the stored U_t(T-1) is zero on both sides
            Ur[-1, ..., 3, :, :] = 0
        self.Ur = Ur
        self.Ar = _blocks_rounded(self.A, self.rnd)
        self.Ainv_r = _blocks_rounded(self.Ainv, self.rnd)
        self.odd = orc.parity_mask(L)

    def scale_hop(self, psi_in):
        """sum over the eight hops of |U|_F |psi(neighbour)| at every site."""
        L = self.L
        nu = np.linalg.norm(self.Ur, axis=(-2, -1))            # [t,z,y,x,mu]
        npsi = np.linalg.norm(psi_in, axis=(-2, -1))           # [t,z,y,x]
        S = np.zeros(npsi.shape)
        for mu in range(4):
            ax = 3 - mu
            S += nu[..., mu] * np.roll(npsi, -1, axis=ax)                     # forward
            S += np.roll(nu[..., mu], 1, axis=ax) * np.roll(npsi, 1, axis=ax)  # backward
        return S


def _check(got, ref, S, u_out, mask, what):
    err = np.abs(got - ref)
    bound = u_out * np.abs(ref) + 64 * 2.0 ** -24 * S[..., None, None]
    bad = (err > bound) & mask[..., None, None]
    worst = float(np.max(np.where(mask[..., None, None], err / np.maximum(bound, 1e-300), 0)))
    print(f"{what}: worst err/bound {worst:.3f}")
    assert not bad.any(), (what, np.argwhere(bad)[:5], err[bad][:5], bound[bad][:5])


@pytest.mark.parametrize("tname,nrhs,tune", TUNINGS, ids=[t[0] for t in TUNINGS])
@pytest.mark.parametrize("prec", [lqcd.F32, lqcd.BF16], ids=["f32", "bf16"])
@pytest.mark.parametrize("c", CASES, ids=case_id)
def test_hop_kernels_per_site(c, prec, tname, nrhs, tune):
    print(f"\n[gpu case] per-site {case_id(c)} prec {prec} {tname}", flush=True)
    s = Case(*c, prec)
    ws = lqcd.Workspace(s.lat, s.pm, nrhs)
    if tune:
        lqcd.set_tuning(ws, prec, **tune)
    psi = np.stack([inputs.gaussian_spinor(s.L, 60 + j, s.bc) for j in range(nrhs)])
    x = torch.from_numpy(psi).cuda()
    got_eo = lqcd.dw_apply(s.gauge, s.d, x, op=lqcd.OP_HOP_EO, prec=prec, ws=ws).cpu().numpy()
    got_oe = lqcd.dw_apply(s.gauge, s.d, x, op=lqcd.OP_HOP_OE, prec=prec, ws=ws).cpu().numpy()
    odd, even = s.odd, ~s.odd
    active = np.ones(odd.shape, bool)
    if s.bc == SF:
        active[0] = False
    nAinv = np.linalg.norm(s.Ainv_r, axis=(-2, -1))
    nA = np.linalg.norm(s.Ar, axis=(-2, -1))
    for j in range(nrhs):
        pr = s.rnd(psi[j])
        if s.bc == SF:
            pr[0] = 0  # the Dirichlet slice is ignored on input
        pe = np.where(even[..., None, None], pr, 0)
        po = np.where(odd[..., None, None], pr, 0)
        # e -> o: A_oo^{-1} D_oe psi_e
        ref = orc.schur_hop_eo(s.L, s.bc, s.theta, s.Ur, s.Ainv_r, pe)
        S = nAinv * s.scale_hop(pe)
        _check(got_eo[j], ref, S, s.u_out, odd & active, f"e->o rhs {j}")
        # o -> e: A_ee x_e - D_eo y_o
        ref = orc.apply_blocks(s.Ar, pe) - orc.hop(s.L, s.bc, s.theta, s.Ur, po)
        S = s.scale_hop(po) + nA * np.linalg.norm(pe, axis=(-2, -1))
        _check(got_oe[j], ref, S, s.u_out, even & active, f"o->e rhs {j}")
        # sites the launch does not produce are zero, and so is the SF slice
        assert not np.any(got_eo[j][even]) and not np.any(got_oe[j][odd])
        if s.bc == SF:
            assert not np.any(got_eo[j][0]) and not np.any(got_oe[j][0])
