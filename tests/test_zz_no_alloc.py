"""The meson contraction entry point that allocates nothing
(lqcd_meson_noalloc, scratch in the library's fixed per-GPU array) against
the workspace entry point lqcd_meson, through the C ABI: two calls in a row
on one GPU, the second on a smaller lattice (so the fixed array still holds
the first call's larger partials), each bit for bit equal to lqcd_meson on
the same input and within 1e-12 of the oracle's contraction."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2503_16994_amd import lqcd

pytestmark = pytest.mark.gpu

PAIRS = [(15, 15), (15, 8), (8, 8), (0, 15), (1, 1)]


def random_columns(L, seed):
    rng = np.random.default_rng(seed)
    shape = (12, L[3], L[2], L[1], L[0], 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_meson_noalloc_equals_the_workspace_entry_point_on_two_calls():
    # 16x16x8x12: 8 chunks per slice x 12 slices; then 6x4x4x6: one ragged chunk
    for L in ((16, 16, 8, 12), (6, 4, 4, 6)):
        print(f"\n[gpu case] meson_noalloc {L}", flush=True)
        psi_h = random_columns(L, seed=11 + sum(L))
        psi = torch.from_numpy(psi_h).cuda()
        lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, (1, 1, 1, -1))
        T = L[3]
        C = torch.full((len(PAIRS), T), float("nan"), dtype=torch.complex128, device="cuda")
        G = torch.full((T, 4, 4, 4, 4), float("nan"), dtype=torch.complex128, device="cuda")
        torch.cuda.synchronize()
        lqcd.meson_noalloc(lat, psi, PAIRS, C, G)
        torch.cuda.synchronize()
        ws = lqcd.Workspace(lat, lqcd.PM_F64, 1)
        C_ws, G_ws = lqcd.meson(lat, psi, PAIRS, ws)
        torch.cuda.synchronize()
        assert torch.equal(C, C_ws) and torch.equal(G, G_ws)
        G_ref = orc.meson_G(L, psi_h)
        assert rel_max(G.cpu().numpy(), G_ref) < 1e-12
        Cg = C.cpu().numpy()
        for p, (m1, m2) in enumerate(PAIRS):
            assert rel_max(Cg[p], orc.meson_correlator(G_ref, m1, m2)) < 1e-12, (L, m1, m2)
        # only the correlators, into caller tensors: the same numbers
        C2 = torch.zeros_like(C)
        lqcd.meson_noalloc(lat, psi, PAIRS, C2, None)
        torch.cuda.synchronize()
        assert torch.equal(C2, C)
        del ws
