"""Plain FP64 CPU oracle for the Wilson-clover operator and its CG solve.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library ``paper_2503_16994_amd`` and never imports it.

The arithmetic lives in ``lqcd_oracle.c`` (see its header for the operator
definition and conventions).  This module loads it with ctypes and adds
the even-odd (Schur complement) pieces as plain compositions of the full
operator, using ``numpy.linalg`` for the 12x12 site-block inverses.

Conventions (paper Sec. 2.1 and Sec. 3.3; the formula itself is the
Sheikholeslami-Wohlert operator the paper cites):

* lattice extents ``L = (Lx, Ly, Lz, T)``, time last;
* canonical arrays: ``U[t, z, y, x, mu, a, b]``, ``psi[t, z, y, x, alpha, a]``;
* ``kappa`` maps to the bare mass ``m0 = 1/(2 kappa) - 4``;
* boundary types ``PERIODIC = 0``, ``SF = 1``, ``OPEN = 2``.

Functions with a pin in ``tests/test_oracle_pins.py``: ``gamma``,
``field_strength``, ``clover_matrix``, ``hop``, ``dw``, ``dw_dag``, ``cg``,
``schur_*``, ``su3_from_two_rows``, ``gamma_product``, ``meson_G``,
``meson_correlator``, ``sf_source``, ``sf_correlators``, ``cg_fixed``,
``singular_extremes``.  None is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

PERIODIC, SF, OPEN = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqcd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP over sites, strict FP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.or_field_strength.argtypes = [P, I, P, P]
        lib.or_clover_matrix.argtypes = [P, I, P, D, D, D, P]
        lib.or_hop.argtypes = [P, I, P, P, P, P, P]
        lib.or_dw.argtypes = [P, I, P, P, P, P, P, P]
        lib.or_dw_dag.argtypes = [P, I, P, P, P, P, P, P]
        lib.or_gamma.argtypes = [I, P]
        lib.or_cg.argtypes = [P, I, P, P, P, P, P, P, D, I, P, P]
        lib.or_cg.restype = I
        lib.or_cg_fixed.argtypes = [P, I, P, P, P, P, P, P, I]
        lib.or_cg_fixed.restype = D
        lib.or_num_threads.restype = I
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _Larr(L):
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32))


def _theta(theta):
    th = np.ones(4, dtype=np.complex128) if theta is None else np.asarray(theta, np.complex128)
    return np.ascontiguousarray(th.real), np.ascontiguousarray(th.imag)


def _c128(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def m0_from_kappa(kappa: float) -> float:
    """Bare mass from the hopping parameter, m0 = 1/(2 kappa) - 4."""
    return 1.0 / (2.0 * kappa) - 4.0


def num_threads() -> int:
    return _load().or_num_threads()


def gamma(mu: int) -> np.ndarray:
    """Chiral-basis gamma matrix (mu = 0..3 for x,y,z,t; 4 for gamma_5)."""
    g = np.zeros((4, 4), np.complex128)
    _load().or_gamma(mu, _ptr(g))
    return g


def field_strength(L, bc, U) -> np.ndarray:
    """Clover field strength F[t,z,y,x,plane,3,3]; planes xy,xz,xt,yz,yt,zt."""
    U = _c128(U)
    Lx, Ly, Lz, T = L
    F = np.zeros((T, Lz, Ly, Lx, 6, 3, 3), np.complex128)
    _load().or_field_strength(_ptr(_Larr(L)), bc, _ptr(U), _ptr(F))
    return F


def clover_matrix(L, bc, U, m0, csw, cF=1.0, mu=0.0) -> np.ndarray:
    """Diagonal term A(x) as 12x12 matrices, A[t,z,y,x,12,12]; with a twisted
    mass mu (paper Sec. 3.3, DiracParam's mu) the site term of
    D(mu) = Dw + i mu g5, i.e. A(x) + i mu g5 (g5 = diag(1,1,-1,-1) on spin,
    identity on colour)."""
    U = _c128(U)
    Lx, Ly, Lz, T = L
    A = np.zeros((T, Lz, Ly, Lx, 12, 12), np.complex128)
    _load().or_clover_matrix(_ptr(_Larr(L)), bc, _ptr(U), m0, csw, cF, _ptr(A))
    if mu != 0.0:
        g5 = np.diag(np.repeat(np.diag(gamma(4)), 3))
        A = A + 1j * mu * g5
    return A


def hop(L, bc, theta, U, psi) -> np.ndarray:
    """Off-diagonal (hopping) part of Dw applied to psi."""
    U, psi = _c128(U), _c128(psi)
    out = np.zeros_like(psi)
    tr, ti = _theta(theta)
    _load().or_hop(_ptr(_Larr(L)), bc, _ptr(tr), _ptr(ti), _ptr(U), _ptr(psi), _ptr(out))
    return out


def dw(L, bc, theta, U, A, psi) -> np.ndarray:
    """Full Wilson-clover operator Dw psi (paper Sec. 3.3, Dw!)."""
    U, A, psi = _c128(U), _c128(A), _c128(psi)
    out = np.zeros_like(psi)
    tr, ti = _theta(theta)
    _load().or_dw(_ptr(_Larr(L)), bc, _ptr(tr), _ptr(ti), _ptr(U), _ptr(A), _ptr(psi), _ptr(out))
    return out


def dw_dag(L, bc, theta, U, A, psi) -> np.ndarray:
    """Dw^+ psi: g5 Dw g5 psi with the site term replaced by g5 A^+ g5 (equal
    to A for the clover term; i mu g5 becomes -i mu g5)."""
    U, A, psi = _c128(U), _c128(A), _c128(psi)
    out = np.zeros_like(psi)
    tr, ti = _theta(theta)
    _load().or_dw_dag(_ptr(_Larr(L)), bc, _ptr(tr), _ptr(ti), _ptr(U), _ptr(A), _ptr(psi), _ptr(out))
    return out


def cg(L, bc, theta, U, A, eta, tol, maxiter=100000):
    """CG on the normal equations (paper Sec. 3.3, CG!/propagator!).

    Returns (psi, rho, iters, converged) with rho the true relative residual
    |eta - Dw psi| / |eta|.
    """
    U, A, eta = _c128(U), _c128(A), _c128(eta)
    psi = np.zeros_like(eta)
    tr, ti = _theta(theta)
    rho = ctypes.c_double(0.0)
    iters = ctypes.c_int(0)
    st = _load().or_cg(_ptr(_Larr(L)), bc, _ptr(tr), _ptr(ti), _ptr(U), _ptr(A), _ptr(eta),
                       _ptr(psi), float(tol), int(maxiter), ctypes.byref(rho), ctypes.byref(iters))
    return psi, rho.value, iters.value, st == 0


def cg_fixed(L, bc, theta, U, A, eta, niter):
    """Exactly ``niter`` CG iterations from zero; returns (psi, |r|/|b|)."""
    U, A, eta = _c128(U), _c128(A), _c128(eta)
    psi = np.zeros_like(eta)
    tr, ti = _theta(theta)
    rel = _load().or_cg_fixed(_ptr(_Larr(L)), bc, _ptr(tr), _ptr(ti), _ptr(U), _ptr(A),
                              _ptr(eta), _ptr(psi), int(niter))
    return psi, rel


# --------------------------------------------------------------------------
# Even-odd pieces, composed from the full operator.
#
# With parity p(x) = (x+y+z+t) mod 2 the operator splits into blocks
#   Dw = [[A_ee, D_eo], [D_oe, A_oo]]
# where A is the site-diagonal term and D the hopping term.  The Schur
# complement on the even sites is  Dhat = A_ee - D_eo A_oo^{-1} D_oe.
# --------------------------------------------------------------------------

def parity_mask(L) -> np.ndarray:
    """Boolean [t,z,y,x] array, True on odd sites."""
    Lx, Ly, Lz, T = L
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return ((x + y + z + t) % 2) == 1


def _restrict(psi, mask):
    out = np.zeros_like(psi)
    out[mask] = psi[mask]
    return out


def apply_blocks(A, psi) -> np.ndarray:
    """Site-diagonal A(x) psi(x)."""
    sh = psi.shape
    v = psi.reshape(sh[:4] + (12,))
    return np.einsum("...rc,...c->...r", A, v).reshape(sh)


def inverse_blocks(A) -> np.ndarray:
    """A(x)^{-1} per site via numpy.linalg.inv on the 12x12 blocks."""
    return np.linalg.inv(A)


def schur_hop_eo(L, bc, theta, U, Ainv, psi_e) -> np.ndarray:
    """A_oo^{-1} D_oe psi_e (input: field supported on even sites)."""
    odd = parity_mask(L)
    h = hop(L, bc, theta, U, _restrict(psi_e, ~odd))
    return _restrict(apply_blocks(Ainv, h), odd)


def schur_dhat(L, bc, theta, U, A, Ainv, psi_e) -> np.ndarray:
    """Dhat psi_e = A_ee psi_e - D_eo A_oo^{-1} D_oe psi_e, even-site output."""
    odd = parity_mask(L)
    pe = _restrict(psi_e, ~odd)
    t = schur_hop_eo(L, bc, theta, U, Ainv, pe)
    out = apply_blocks(A, pe) - hop(L, bc, theta, U, t)
    out = _restrict(out, ~odd)
    if bc == SF:
        out[0] = 0.0
    return out


def schur_source(L, bc, theta, U, Ainv, eta) -> np.ndarray:
    """eta_hat_e = eta_e - D_eo A_oo^{-1} eta_o."""
    odd = parity_mask(L)
    t = _restrict(apply_blocks(Ainv, _restrict(eta, odd)), odd)
    out = _restrict(eta, ~odd) - _restrict(hop(L, bc, theta, U, t), ~odd)
    if bc == SF:
        out[0] = 0.0
    return out


def schur_reconstruct(L, bc, theta, U, Ainv, eta, psi_e) -> np.ndarray:
    """psi = psi_e + A_oo^{-1} (eta_o - D_oe psi_e) on the odd sites."""
    odd = parity_mask(L)
    pe = _restrict(psi_e, ~odd)
    rhs = _restrict(eta, odd) - _restrict(hop(L, bc, theta, U, pe), odd)
    po = _restrict(apply_blocks(Ainv, rhs), odd)
    out = pe + po
    if bc == SF:
        out[0] = 0.0
    return out


def su3_from_two_rows(U2) -> np.ndarray:
    """Links ``U[..., 3, 3]`` from their first two rows ``U2[..., 2, 3]``.

    Paper Sec. 2.2: the SU(3) element type stores two rows; the third follows
    from U^-1 = U^+ and det U = 1.  Together these make U^+ the adjugate of U,
    so every entry of row 2 is the complex conjugate of its cofactor, which is
    built from rows 0 and 1 alone: row 2 = conj(row 0 x row 1).  (For a
    unitary U of determinant d the same formula gives conj(d) times row 2.)"""
    U2 = np.asarray(U2, np.complex128)
    r0, r1 = U2[..., 0, :], U2[..., 1, :]
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def gamma_product(mask: int) -> np.ndarray:
    """Gamma_m = g_t^{m3} g_x^{m0} g_y^{m1} g_z^{m2}, the ordered product with
    g_t first (mask 15 is g5 = g_t g_x g_y g_z, 0 the identity)."""
    out = np.eye(4, dtype=np.complex128)
    for mu in (3, 0, 1, 2):
        if (mask >> mu) & 1:
            out = out @ gamma(mu)
    return out


def meson_G(L, psi12) -> np.ndarray:
    """Colour-traced spin tensor of a 12-column point-source propagator per
    time slice (paper Sec. 3.3: correlators contracted from propagators):
    G[t, al, be, al', be'] = sum_{x in slice t} sum_{a, c} S(x)[al a][be c] conj(S(x)[al' a][be' c]),
    with S(x)[al a][be c] = psi12[3 be + c][x][al][a] (column 3 s + c: source
    spin s, colour c)."""
    Lx, Ly, Lz, T = L
    P = np.asarray(psi12, np.complex128).reshape(4, 3, T, Lz * Ly * Lx, 4, 3)  # [be, c, t, x, al, a]
    return np.einsum("bctxAa,dctxBa->tAbBd", P, P.conj())


def meson_correlator(G, m1: int, m2: int) -> np.ndarray:
    """C[t] = sum_x tr[Gamma_m1 S(x) Gamma_m2 g5 S(x)^+ g5] (backward
    propagator from g5-hermiticity), written with G:
    sum Gamma[de][al] Gamma'[be][ga] g5[ga] g5[de] G[t][al][be][de][ga]."""
    A, B = gamma_product(m1), gamma_product(m2)
    g5 = np.diag(gamma(4)).real
    return np.einsum("da,bg,g,d,tabdg->t", A, B, g5, g5, G)


def sf_source(L, U) -> np.ndarray:
    """Boundary source of the Schroedinger-functional boundary-to-bulk
    propagator (paper Sec. 3.3): the 12 columns (s, c) of P+ U_t(0, y)^+ on
    the slice y0 = 1, P+ = (1 + g_t)/2, i.e.
    eta_{3s+c}(y)[al][a] = delta_{y0,1} P+[al][s] conj(U_t(y0 = 0, y)[c][a])."""
    Lx, Ly, Lz, T = L
    Pp = (np.eye(4) + gamma(3)) / 2
    eta = np.zeros((12, T, Lz, Ly, Lx, 4, 3), np.complex128)
    Ut0 = np.asarray(U)[0, :, :, :, 3]  # [z, y, x, c, a]: the link from y0 = 0 to y0 = 1
    for s in range(4):
        for c in range(3):
            eta[3 * s + c, 1] = Pp[:, s][None, None, None, :, None] * np.conj(Ut0[:, :, :, c, :])[:, :, :, None, :]
    return eta


def sf_correlators(L, H):
    """f_P(x0) = 1/2 sum_x tr[H(x)^+ H(x)] and f_A(x0) = -1/2 sum_x tr[H(x)^+ g_t H(x)]
    of the boundary-to-bulk propagator H (12 columns, H(x)[al a][s c] =
    H_{3s+c}(x)[al][a], the solution for `sf_source`)."""
    Lx, Ly, Lz, T = L
    Hm = np.asarray(H, np.complex128).reshape(12, T, Lx * Ly * Lz, 4, 3)  # [col, t, x, al, a]
    fP = 0.5 * np.einsum("jtxAa,jtxAa->t", Hm.conj(), Hm)
    fA = -0.5 * np.einsum("jtxAa,AB,jtxBa->t", Hm.conj(), gamma(3), Hm)
    return fP, fA


def singular_extremes(L, bc, theta, U, A, seed=0, max_steps=300, rtol=1e-7, solve_tol=1e-12,
                      op="full", want_max=True):
    """Largest and smallest singular value of Dw on its active sites (every
    site; with SF boundaries the slice t = 0 is excluded: the operator maps
    it to zero and ignores it), or with op="schur" of the even-odd Schur
    complement Dhat = A_ee - D_eo A_oo^{-1} D_oe on the active even sites,
    for the error bound of a solve (|psi - psi_exact| / |psi_exact| <=
    cond * rho with rho the true relative residual) and for the conditioning
    of the normal equations (cond(D^+ D) = cond(D)^2).

    sigma_max: power iteration on D^+ D (skipped with want_max=False: 0 is
    returned); sigma_min: inverse iteration on D^+ D, each step
    x = D^{-1} g5 D^{-1} g5 v (D^{-+} = g5 D^{-1} g5 for both operators).
    Dw^{-1} is the oracle's CG to solve_tol; Dhat^{-1} v_e is the even part of
    Dw^{-1} (v_e, 0) (block elimination of the odd sites).  Both iterations
    stop when the Rayleigh quotient changes by less than rtol relative.
    Returns (sigma_max, sigma_min, steps_max, steps_min); the inverse
    iteration's sigma_min is an upper bound on the true one.
    """
    Lx, Ly, Lz, T = L
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (T, Lz, Ly, Lx, 4, 3)
    odd = parity_mask(L)
    schur = (op == "schur")
    Ainv = inverse_blocks(A) if schur else None

    def start():
        v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        if bc == SF:
            v[0] = 0
        if schur:
            v[odd] = 0
        return v / np.linalg.norm(v)

    def g5(v):
        w = v.copy()
        w[..., 2:, :] *= -1
        return w

    def fwd(v):
        return schur_dhat(L, bc, theta, U, A, Ainv, v) if schur else dw(L, bc, theta, U, A, v)

    def inv(v):
        x = cg(L, bc, theta, U, A, v, solve_tol)[0]
        return _restrict(x, ~odd) if schur else x

    lam, steps_max = 0.0, 0
    if want_max:
        v = start()
        for steps_max in range(1, max_steps + 1):
            w = g5(fwd(g5(fwd(v))))  # D^+ D v
            new = float(np.vdot(v, w).real)  # |D v|^2
            v = w / np.linalg.norm(w)
            if abs(new - lam) <= rtol * new:
                lam = new
                break
            lam = new
    v = start()
    mu, steps_min = 0.0, 0
    for steps_min in range(1, max_steps + 1):
        z = g5(inv(g5(v)))  # D^{-+} v
        x = inv(z)          # (D^+ D)^{-1} v
        new = float(np.vdot(z, z).real)  # v^+ (D^+ D)^{-1} v
        v = x / np.linalg.norm(x)
        if abs(new - mu) <= rtol * new:
            mu = new
            break
        mu = new
    return float(np.sqrt(lam)), float(1.0 / np.sqrt(mu)), steps_max, steps_min


def dense_dw(L, bc, theta, U, A) -> np.ndarray:
    """Dw as a dense (12V x 12V) matrix, column j = Dw e_j (tiny lattices)."""
    Lx, Ly, Lz, T = L
    n = Lx * Ly * Lz * T * 12
    M = np.zeros((n, n), np.complex128)
    e = np.zeros((T, Lz, Ly, Lx, 4, 3), np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[j] = 1.0
        M[:, j] = dw(L, bc, theta, U, A, e).reshape(-1)
        flat[j] = 0.0
    return M
