"""Seeded synthetic inputs: gauge fields and sources.

This module is shared by the tests, the benchmark and the smoke check, and
serves both the GPU path and the CPU oracle.  It holds none of the
operator's arithmetic: it only draws random numbers and builds fields in the
canonical layout

* ``U[t, z, y, x, mu, a, b]`` (complex128), mu = 0..3 = x, y, z, t;
* ``psi[t, z, y, x, alpha, a]`` (complex128), alpha = spin, a = colour.

Recipe (the paper's workloads use HMC-generated SU(3) ensembles, which are
not available here; these seeded fields stand in for them):

* links ``U = exp(i eps H)`` with ``H = sum_a h_a lambda_a / 2`` traceless
  Hermitian, ``h_a ~ N(0, 1)`` i.i.d. (lambda_a the Gell-Mann matrices),
  drawn in canonical order (site, mu, a) from ``numpy`` ``PCG64(seed)``;
  the exponential is taken by eigendecomposition, so ``det U = 1``;
* for Schroedinger-functional boundaries the spatial links on slice t = 0
  are replaced by the constant boundary field
  ``diag(exp(i phi1/L_k), exp(i phi2/L_k), exp(-i(phi1+phi2)/L_k))``
  (paper Sec. 3.1, the GaugeParm paragraph);
* point sources ``eta = delta_{x,x0} delta_{alpha,s} delta_{a,c}``;
* Z2 complex noise, every component ``(+-1 +- i)/sqrt(2)`` independently.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

PERIODIC, SF, OPEN = 0, 1, 2


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return lam


def volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def gauge_field(L, eps: float, seed: int, bc: int = PERIODIC, sf_phi=(0.0, 0.0),
                chunk: int = 1 << 18) -> np.ndarray:
    """SU(3) links U = exp(i eps H), H Gaussian traceless Hermitian."""
    Lx, Ly, Lz, T = (int(v) for v in L)
    V = volume(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = _gell_mann() / 2.0
    U = np.empty((V * 4, 3, 3), np.complex128)
    n = V * 4
    # the draws are sequential (reproducible); the exponentials of the chunks
    # are independent and run on a thread pool (LAPACK releases the GIL)
    chunks = []
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        chunks.append((s, m, rng.standard_normal((m, 8))))

    def expo(item):
        s, m, h = item
        H = np.einsum("na,aij->nij", h, lam)
        w, v = np.linalg.eigh(H)
        U[s:s + m] = np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())

    workers = min(len(chunks), max(1, min(16, os.cpu_count() or 1)))
    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(expo, chunks))
    else:
        for item in chunks:
            expo(item)
    U = U.reshape(T, Lz, Ly, Lx, 4, 3, 3)
    if bc == SF:
        phi1, phi2 = sf_phi
        for k, Lk in enumerate((Lx, Ly, Lz)):
            d = np.exp(1j * np.array([phi1, phi2, -(phi1 + phi2)]) / Lk)
            U[0, :, :, :, k] = np.diag(d)
    return U


def unit_gauge(L) -> np.ndarray:
    Lx, Ly, Lz, T = (int(v) for v in L)
    U = np.zeros((T, Lz, Ly, Lx, 4, 3, 3), np.complex128)
    U[..., :, :] = np.eye(3)
    return U


def point_source(L, x0=(0, 0, 0, 0), spin: int = 0, colour: int = 0) -> np.ndarray:
    Lx, Ly, Lz, T = (int(v) for v in L)
    eta = np.zeros((T, Lz, Ly, Lx, 4, 3), np.complex128)
    x, y, z, t = x0
    eta[t, z, y, x, spin, colour] = 1.0
    return eta


def point_sources_12(L, x0=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 spin-colour point sources at x0, column j = 3*spin + colour."""
    return np.stack([point_source(L, x0, j // 3, j % 3) for j in range(12)])


def z2_noise(L, seed: int, bc: int = PERIODIC) -> np.ndarray:
    Lx, Ly, Lz, T = (int(v) for v in L)
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2, size=(T, Lz, Ly, Lx, 4, 3, 2))
    sgn = 1.0 - 2.0 * bits
    eta = (sgn[..., 0] + 1j * sgn[..., 1]) / np.sqrt(2.0)
    if bc == SF:
        eta[0] = 0.0
    return eta


def gaussian_spinor(L, seed: int, bc: int = PERIODIC) -> np.ndarray:
    """Complex Gaussian spinor field (test vectors)."""
    Lx, Ly, Lz, T = (int(v) for v in L)
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((T, Lz, Ly, Lx, 4, 3, 2))
    eta = v[..., 0] + 1j * v[..., 1]
    if bc == SF:
        eta[0] = 0.0
    return eta
