"""Pins of the oracle's three-dimensional tensor-product path.

The 3D potential stencil is pinned to independent 1D assemblies (a
separable potential is the Kronecker sum of 1D potential matrices), the
operator to dense Kronecker products built with NumPy, the generalised
spectrum to the isotropic harmonic oscillator (3/2, 5/2 three times, ...),
the Crank-Nicolson step to a dense direct solve and to the exact Cayley
phase of a separable eigenstate, and the propagation to norm conservation.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_18472_amd import workloads as W


def kron3(az, ay, ax):
    return np.kron(az, np.kron(ay, ax))


def tiny(order=4, n=(9, 8, 7), L=(5.0, 4.5, 4.0)):
    bx = W.breaks_uniform(L[0], n[0])
    by = W.breaks_symexp(L[1], n[1], 0.8)
    bz = W.breaks_uniform(L[2], n[2])
    return bx, by, bz, order


def dense_of(m3, V3=None, Ebar=0.0):
    D = {k: O.band_to_dense(m3[k]) for k in ("Sx", "Tx", "Dx", "Sy", "Ty", "Sz", "Tz")}
    S3 = kron3(D["Sz"], D["Sy"], D["Sx"])
    H3 = (kron3(D["Sz"], D["Sy"], D["Tx"]) + kron3(D["Sz"], D["Ty"], D["Sx"]) + kron3(D["Tz"], D["Sy"], D["Sx"])
          + Ebar * kron3(D["Sz"], D["Sy"], D["Dx"]))
    if V3 is not None:
        Nx, Ny, Nz, p = m3["Nx"], m3["Ny"], m3["Nz"], m3["p"]
        n = Nx * Ny * Nz
        Vd = np.zeros((n, n))
        for row in range(n):
            iz, rem = divmod(row, Ny * Nx)
            iy, ix = divmod(rem, Nx)
            for dz in range(-p, p + 1):
                for dy in range(-p, p + 1):
                    for dx in range(-p, p + 1):
                        jz, jy, jx = iz + dz, iy + dy, ix + dx
                        if 0 <= jz < Nz and 0 <= jy < Ny and 0 <= jx < Nx:
                            Vd[row, (jz * Ny + jy) * Nx + jx] = V3[row, dz + p, dy + p, dx + p]
        H3 = H3 + Vd
    return S3, H3


def test_separable_potential_is_the_kronecker_sum_of_1d_matrices():
    bx, by, bz, order = tiny()
    f, g, h = (lambda x: 0.3 * x * x - x), (lambda y: np.cos(y)), (lambda z: 0.5 * z)
    m3 = O.assemble_3d(bx, by, bz, order, 6, lambda x, y, z: f(x) + g(y) + h(z))
    Vx = O.band_to_dense(O.assemble(bx, order, 6, V=f)["V"])
    Vy = O.band_to_dense(O.assemble(by, order, 6, V=g)["V"])
    Vz = O.band_to_dense(O.assemble(bz, order, 6, V=h)["V"])
    Sx, Sy, Sz = (O.band_to_dense(m3[k]) for k in ("Sx", "Sy", "Sz"))
    ref = kron3(Sz, Sy, Vx) + kron3(Sz, Vy, Sx) + kron3(Vz, Sy, Sx)
    S3, H3 = dense_of(m3, m3["V3"])
    S3b, H3b = dense_of(m3)
    got = H3 - H3b
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    # symmetric, and the stencil of a row sits at the right neighbours
    assert np.abs(got - got.T).max() < 1e-14 * np.abs(got).max()


def test_apply_3d_matches_dense_products():
    bx, by, bz, order = tiny()
    m3 = O.assemble_3d(bx, by, bz, order, 5, lambda x, y, z: -1.0 / np.sqrt(x * x + y * y + z * z + 1.0))
    rng = np.random.default_rng(1)
    n = m3["Nx"] * m3["Ny"] * m3["Nz"]
    c = rng.normal(size=n) + 1j * rng.normal(size=n)
    a, b, Eb = 0.7 - 0.2j, 0.3 + 1.1j, 0.37
    S3, H3 = dense_of(m3, m3["V3"], Eb)
    ref = a * (S3 @ c) + b * (H3 @ c)
    got = O.apply_3d(m3, c, a, b, Eb)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_isotropic_oscillator_levels():
    """V = r^2 / 2 on a tensor basis: the generalised eigenvalues of (H3, S3)
    are the sorted sums of three 1D eigenvalues of the same basis (exact up
    to rounding), and the lowest sit at the 3D oscillator levels 3/2, 5/2
    (three times) to the basis error."""
    import itertools
    import scipy.linalg as sl
    order = 5
    b = W.breaks_uniform(6.0, 14)
    m3 = O.assemble_3d(b, b, b, order, 8, lambda x, y, z: 0.5 * (x * x + y * y + z * z))
    S3, H3 = dense_of(m3, m3["V3"])
    ev = sl.eigh(H3, S3, eigvals_only=True, subset_by_index=[0, 9])
    Sx = O.band_to_dense(m3["Sx"])
    Hx = O.band_to_dense(m3["Tx"]) + O.band_to_dense(O.assemble(b, order, 8, V=lambda x: 0.5 * x * x)["V"])
    e1 = sl.eigh(Hx, Sx, eigvals_only=True)[:6]
    sums = np.sort([a + b_ + c for a, b_, c in itertools.product(e1, e1, e1)])[:10]
    assert np.abs(ev - sums).max() < 1e-10
    assert np.abs(ev[:4] - np.array([1.5, 2.5, 2.5, 2.5])).max() < 2e-3


def test_cn_step_matches_dense_solve_and_norm_is_conserved():
    bx, by, bz, order = tiny()
    m3 = O.assemble_3d(bx, by, bz, order, 5, lambda x, y, z: -1.0 / np.sqrt(x * x + y * y + z * z + 1.0))
    n = m3["Nx"] * m3["Ny"] * m3["Nz"]
    rng = np.random.default_rng(2)
    c = rng.normal(size=n) + 1j * rng.normal(size=n)
    alpha, Eb = 0.03, 0.2
    S3, H3 = dense_of(m3, m3["V3"], Eb)
    rhs = (S3 - 1j * alpha * H3) @ c
    ref = np.linalg.solve(S3 + 1j * alpha * H3, rhs)
    got, its = O.cn_solve_3d(m3, rhs, alpha, Eb, tol=1e-14)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    E = 0.1 * np.sin(0.4 * np.arange(11))
    obs, cf = O.propagate_3d(m3, c, E, 0.06, 10)
    assert np.abs(obs[:, 0] / obs[0, 0] - 1.0).max() < 1e-12


def test_separable_eigenstate_takes_the_cayley_phase():
    order = 4
    b = W.breaks_uniform(6.0, 10)
    V1 = lambda x: 0.5 * x * x
    m3 = O.assemble_3d(b, b, b, order, 6, lambda x, y, z: V1(x) + V1(y) + V1(z))
    m1 = O.assemble(b, order, 6, V=V1)
    ev, vec = O.eig_banded(m1["H0"], m1["S"], 2, -0.1)
    c0 = np.einsum("z,y,x->zyx", vec[0], vec[1], vec[0]).reshape(-1).astype(np.complex128)
    eps = 2 * ev[0] + ev[1]
    ns, dt = 12, 0.1
    obs, cf = O.propagate_3d(m3, c0, np.zeros(ns + 1), dt, ns, tol=1e-15)
    a = 0.5 * dt
    ph = ((1 - 1j * a * eps) / (1 + 1j * a * eps)) ** ns
    assert np.abs(cf.reshape(-1) - ph * c0).max() < 1e-11
    assert np.abs(cf.reshape(-1) - np.conj(ph) * c0).max() > 1e-3


def test_v3_rows_from_the_definition_match_the_factorised_assembly():
    """Two independent routes to V3: the C assembly (sum-factorised per span
    triple) and the direct quadrature sum per row (v3_rows)."""
    bx, by, bz, order = tiny()
    V = lambda x, y, z: -1.0 / np.sqrt(x * x + 0.5 * y * y + 2.0 * z * z + 0.3) + 0.1 * x * z
    m3 = O.assemble_3d(bx, by, bz, order, 5, V)
    n = m3["Nx"] * m3["Ny"] * m3["Nz"]
    rows = np.r_[0, 1, m3["Nx"] - 1, n // 2, n // 3 + 7, n - m3["Nx"], n - 1]
    got = O.v3_rows(bx, by, bz, order, 5, V, rows)
    ref = m3["V3"][rows]
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_apply_rows_match_the_operator():
    bx, by, bz, order = tiny()
    V = lambda x, y, z: -1.0 / np.sqrt(x * x + y * y + z * z + 1.0)
    m3 = O.assemble_3d(bx, by, bz, order, 5, V)
    n = m3["Nx"] * m3["Ny"] * m3["Nz"]
    rng = np.random.default_rng(4)
    c = rng.normal(size=n) + 1j * rng.normal(size=n)
    rows = np.r_[0, 5, n // 2, n - 1, rng.integers(0, n, 6)]
    a, b, Eb = 0.4 + 0.1j, -0.2 + 0.9j, 0.21
    got = O.apply_3d_rows(m3, O.v3_rows(bx, by, bz, order, 5, V, rows), rows, c, a, b, Eb)
    ref = O.apply_3d(m3, c, a, b, Eb)[rows]
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
