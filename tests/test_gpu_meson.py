"""GPU parity of the meson contraction (lqcd_meson) against the oracle's
meson_G / meson_correlator, on the same seeded 12-column fields.

Tolerance: relative 1e-12 (max-norm over the tensor, resp. over each
correlator): both sides sum the same FP64 products, in different orders,
over at most a few thousand sites per slice.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_16994_amd import inputs, lqcd

pytestmark = pytest.mark.gpu

# every diagonal pair and a few mixed ones (g5 with g_t, 1 with g5, g_x with g_y)
PAIRS = [(m, m) for m in range(16)] + [(15, 8), (0, 15), (1, 2)]


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def random_columns(L, seed):
    rng = np.random.default_rng(seed)
    shape = (12, L[3], L[2], L[1], L[0], 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# 6x4x4x6: V3 = 96 (one partial chunk); 12x10x8x6: V3 = 960 = 3 x 256 + 192
# (ragged last chunk); 16x16x8x4: V3 = 2048 (eight full chunks)
@pytest.mark.parametrize("L", [(6, 4, 4, 6), (12, 10, 8, 6), (16, 16, 8, 4)], ids=lambda L: "x".join(map(str, L)))
def test_meson_matches_oracle_on_random_columns(L):
    print(f"\n[gpu case] meson {L}", flush=True)
    psi = random_columns(L, seed=sum(L))
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, (1, 1, 1, -1))
    ws = lqcd.Workspace(lat, lqcd.PM_F64, 1)
    C, G = lqcd.meson(lat, torch.from_numpy(psi).cuda(), PAIRS, ws)
    torch.cuda.synchronize()
    G_ref = orc.meson_G(L, psi)
    assert rel_max(G.cpu().numpy(), G_ref) < 1e-12
    Cg = C.cpu().numpy()
    for p, (m1, m2) in enumerate(PAIRS):
        ref = orc.meson_correlator(G_ref, m1, m2)
        assert rel_max(Cg[p], ref) < 1e-12, (m1, m2)
    # only C, then only G: the same numbers
    C2, none = lqcd.meson(lat, torch.from_numpy(psi).cuda(), PAIRS[:3], ws, want_G=False)
    assert none is None and np.array_equal(C2.cpu().numpy(), Cg[:3])
    none, G2 = lqcd.meson(lat, torch.from_numpy(psi).cuda(), [], ws)
    assert none is None and np.array_equal(G2.cpu().numpy(), G.cpu().numpy())


def test_meson_of_a_solved_propagator():
    """12 point sources solved by lqcd_solve (8^3x16, FP64 eo-CG, two-row
    links), contracted on the GPU: equal to the oracle's contraction of the
    same solution; the pion correlator is positive."""
    L = (8, 8, 8, 16)
    U = inputs.gauge_field(L, 0.2, seed=7)
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, (1, 1, 1, -1))
    g = lqcd.GaugeField(lat, torch.from_numpy(U), lqcd.PM_F64 | lqcd.PM_TWO_ROW)
    eta = torch.from_numpy(inputs.point_sources_12(L, (0, 0, 0, 0))).cuda()
    ws = lqcd.Workspace(lat, lqcd.PM_F64, 12)
    r = lqcd.solve(g, eta, 0.1345, 1.9, tol=1e-10, ws=ws)
    assert r.status == lqcd.OK
    C, G = lqcd.meson(lat, r.psi, PAIRS, ws)
    torch.cuda.synchronize()
    psi = r.psi.cpu().numpy()
    G_ref = orc.meson_G(L, psi)
    assert rel_max(G.cpu().numpy(), G_ref) < 1e-12
    pion = C.cpu().numpy()[15]
    assert rel_max(pion, orc.meson_correlator(G_ref, 15, 15)) < 1e-12
    assert np.all(pion.real > 0) and np.max(np.abs(pion.imag)) < 1e-10 * np.max(pion.real)
    print("pion correlator:", np.array2string(pion.real, precision=4))


def test_meson_full_size_sampled_slices():
    """32^3x64 (the C3 lattice), random columns: the GPU contraction over the
    whole lattice, checked on four time slices against the oracle on those
    slices alone."""
    L = (32, 32, 32, 64)
    rng = np.random.default_rng(5)
    shape = (12, 64, 32, 32, 32, 4, 3)
    psi = torch.complex(torch.randn(shape, dtype=torch.float64, device="cuda"),
                        torch.randn(shape, dtype=torch.float64, device="cuda"))
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, (1, 1, 1, -1))
    ws = lqcd.Workspace(lat, lqcd.PM_F64, 1)
    C, G = lqcd.meson(lat, psi, [(15, 15), (8, 8)], ws)
    torch.cuda.synchronize()
    Gg, Cg = G.cpu().numpy(), C.cpu().numpy()
    for t in sorted(rng.choice(64, 4, replace=False)):
        sl = psi[:, t:t + 1].cpu().numpy()
        G_ref = orc.meson_G((32, 32, 32, 1), sl)[0]
        assert rel_max(Gg[t], G_ref) < 1e-12, t
        assert abs(Cg[0, t] - orc.meson_correlator(G_ref[None], 15, 15)[0]) < 1e-12 * abs(Cg[0, t])
    del psi
    torch.cuda.empty_cache()
