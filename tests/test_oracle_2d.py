"""Pins for the oracle's two-dimensional tensor-product path: potential
stencil, operator application, Crank-Nicolson solve and propagation.

Each check is against something the 2D code does not share: 1D assemblies
combined by Kronecker products (exact for separable potentials), dense
direct linear algebra on tiny grids, the harmonic-oscillator spectrum and the
exact Cayley phase of a separable eigenstate."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import oracle as O
from paper_2608_18472_amd import workloads as W


def dense(band):
    return O.band_to_dense(band)


def dense_2d(m2, Ebar=0.0, with_V=True):
    """S2 and H2 as dense matrices from 1D Kronecker products (row-major
    index iy*Nx + ix) plus the potential stencil."""
    Sx, Tx, Dx = dense(m2["Sx"]), dense(m2["Tx"]), dense(m2["Dx"])
    Sy, Ty = dense(m2["Sy"]), dense(m2["Ty"])
    S2 = np.kron(Sy, Sx)
    H2 = np.kron(Sy, Tx) + np.kron(Ty, Sx) + Ebar * np.kron(Sy, Dx)
    if with_V:
        Nx, Ny, p = m2["Nx"], m2["Ny"], m2["p"]
        V = np.zeros_like(S2)
        for iy in range(Ny):
            for ix in range(Nx):
                for dy in range(-p, p + 1):
                    for dx in range(-p, p + 1):
                        jy, jx = iy + dy, ix + dx
                        if 0 <= jy < Ny and 0 <= jx < Nx:
                            V[iy * Nx + ix, jy * Nx + jx] = m2["V2"][iy * Nx + ix, dy + p, dx + p]
        H2 = H2 + V
    return S2, H2


def test_separable_potential_is_the_kronecker_sum_of_1d_potentials():
    bx = W.breaks_symexp(6.0, 11, 1.5)
    by = np.linspace(-4.0, 5.0, 9)
    order, nq = 5, 8
    f = lambda x: x * x - 0.3 * x
    g = lambda y: np.cos(y)
    m2 = O.assemble_2d(bx, by, order, nq, lambda x, y: f(x) + g(y))
    mx = O.assemble(bx, order, nq, V=f)
    my = O.assemble(by, order, nq, V=g)
    Vx, Sx, Vy, Sy = dense(mx["V"]), dense(mx["S"]), dense(my["V"]), dense(my["S"])
    Nx, Ny, p = m2["Nx"], m2["Ny"], m2["p"]
    err = 0.0
    for iy in range(Ny):
        for ix in range(Nx):
            for dy in range(-p, p + 1):
                for dx in range(-p, p + 1):
                    jy, jx = iy + dy, ix + dx
                    want = 0.0
                    if 0 <= jy < Ny and 0 <= jx < Nx:
                        want = Vx[ix, jx] * Sy[iy, jy] + Sx[ix, jx] * Vy[iy, jy]
                    err = max(err, abs(m2["V2"][iy * Nx + ix, dy + p, dx + p] - want))
    assert err < 1e-13 * np.abs(m2["V2"]).max()


def test_apply_matches_dense_operator():
    bx = np.linspace(-3.0, 3.0, 8)
    by = W.breaks_symexp(4.0, 7, 1.2)
    m2 = O.assemble_2d(bx, by, 4, 6, lambda x, y: -1.0 / np.sqrt(x * x + y * y + 1.0))
    rng = np.random.default_rng(1)
    c = rng.normal(size=m2["Nx"] * m2["Ny"]) + 1j * rng.normal(size=m2["Nx"] * m2["Ny"])
    a, b, Eb = 0.7 - 0.2j, 0.3 + 1.1j, 0.37
    S2, H2 = dense_2d(m2, Eb)
    want = a * (S2 @ c) + b * (H2 @ c)
    got = O.apply_2d(m2, c, a, b, Eb)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_cn_solve_matches_dense_direct_solve():
    bx = np.linspace(-3.0, 3.0, 7)
    by = np.linspace(-2.5, 2.0, 6)
    m2 = O.assemble_2d(bx, by, 4, 6, lambda x, y: -1.0 / np.sqrt(x * x + y * y + 1.0))
    alpha, Eb = 0.04, 0.8
    S2, H2 = dense_2d(m2, Eb)
    rng = np.random.default_rng(2)
    rhs = rng.normal(size=S2.shape[0]) + 1j * rng.normal(size=S2.shape[0])
    want = np.linalg.solve(S2 + 1j * alpha * H2, rhs)
    got, its = O.cn_solve_2d(m2, rhs, alpha, Eb, tol=1e-15)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    assert its < 60


def test_2d_harmonic_oscillator_levels():
    """Lowest levels 1, 2, 2, 3, 3, 3 of V = (x^2 + y^2)/2; the error is the
    discretisation error (5e-8 here, 3e-11 with 41 breakpoints at order 8)."""
    br = np.linspace(-7.0, 7.0, 31)
    m2 = O.assemble_2d(br, br, 7, 8, lambda x, y: 0.5 * (x * x + y * y))
    S2, H2 = dense_2d(m2)
    ev = sl.eigh(H2, S2, eigvals_only=True)[:6]
    assert np.abs(ev - np.array([1.0, 2.0, 2.0, 3.0, 3.0, 3.0])).max() < 1e-7


def test_separable_eigenstate_has_the_exact_cayley_phase():
    """Zero field, separable potential: the product of 1D generalised
    eigenvectors is an eigenvector of the 2D pencil with eps = eps_x + eps_y,
    so n CN steps multiply it by ((1 - i a eps)/(1 + i a eps))^n."""
    br = np.linspace(-6.0, 6.0, 14)
    order, nq, dt, ns = 5, 8, 0.1, 25
    m2 = O.assemble_2d(br, br, order, nq, lambda x, y: 0.5 * x * x + 0.7 * y * y)
    mx = O.assemble(br, order, nq, V=lambda x: 0.5 * x * x)
    my = O.assemble(br, order, nq, V=lambda y: 0.7 * y * y)
    ex, vx = O.eig_banded(mx["T"] + mx["V"], mx["S"], 1, 0.0)
    ey, vy = O.eig_banded(my["T"] + my["V"], my["S"], 1, 0.0)
    psi0 = np.outer(vy[0], vx[0]).astype(np.complex128)
    eps = ex[0] + ey[0]
    a = 0.5 * dt
    obs, c = O.propagate_2d(m2, psi0, np.zeros(ns + 1), dt, ns)
    ph = ((1 - 1j * a * eps) / (1 + 1j * a * eps)) ** ns
    assert np.abs(c - ph * psi0).max() < 1e-11
    assert np.abs(obs[:, 0] - 1.0).max() < 1e-12


def test_norm_is_conserved_under_the_field():
    bx = np.linspace(-8.0, 8.0, 13)
    by = np.linspace(-7.0, 7.0, 11)
    m2 = O.assemble_2d(bx, by, 4, 6, lambda x, y: -1.0 / np.sqrt(x * x + y * y + 1.0))
    rng = np.random.default_rng(3)
    psi0 = rng.normal(size=(m2["Ny"], m2["Nx"])) + 1j * rng.normal(size=(m2["Ny"], m2["Nx"]))
    E = 0.3 * np.sin(0.4 * np.arange(31))
    obs, _ = O.propagate_2d(m2, psi0, E, 0.1, 30)
    assert np.abs(obs[:, 0] / obs[0, 0] - 1.0).max() < 1e-12


def test_stencil_apply_matches_dense_stencil_matrix():
    """The oracle's offset-sum product with a stencil (used for the
    acceleration) equals the dense matrix built entry by entry."""
    bx = np.linspace(-3.0, 3.0, 9)
    by = W.breaks_symexp(4.0, 8, 1.1)
    m2 = O.assemble_2d(bx, by, 5, 6, lambda x, y: -1.0 / np.sqrt(x * x + y * y + 1.0),
                       dVx=lambda x, y: x / (x * x + y * y + 1.0) ** 1.5)
    rng = np.random.default_rng(7)
    n = m2["Nx"] * m2["Ny"]
    c = rng.normal(size=n) + 1j * rng.normal(size=n)
    for key in ("V2", "G2"):
        mk = dict(m2, V2=m2[key])
        S2, H2 = dense_2d(mk)
        _, H0 = dense_2d(mk, with_V=False)
        ref = (H2 - H0) @ c
        got = O.stencil_apply_2d(m2, m2[key], c)
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max(), key


def test_force_stencil_of_the_oscillator_is_the_dipole_matrix():
    """V = (x^2 + y^2)/2 has dV/dx = x: the stencil of dV/dx (2D quadrature)
    equals D2 = Dx (x) Sy from the 1D assemblies, so the acceleration of a
    field-free oscillator is -d (and -d - E nu with a field)."""
    bx = W.breaks_symexp(5.0, 10, 1.3)
    by = np.linspace(-4.0, 4.5, 9)
    m2 = O.assemble_2d(bx, by, 4, 7, lambda x, y: 0.5 * (x * x + y * y), dVx=lambda x, y: x + 0.0 * y)
    Dx, Sy = dense(m2["Dx"]), dense(m2["Sy"])
    D2 = np.kron(Sy, Dx)
    _, H2a = dense_2d(dict(m2, V2=m2["G2"]))
    _, H0 = dense_2d(m2, with_V=False)
    G2 = H2a - H0
    assert np.abs(G2 - D2).max() < 1e-12 * np.abs(D2).max()


def test_acceleration_is_the_second_derivative_of_the_dipole():
    """Ehrenfest for constant mass (section IV.A): d''(t) = a(t) =
    -<dV/dx> - E <1> in the complete-basis limit.  For a driven ground state
    the second difference of the propagated dipole meets the acceleration
    column to 1e-4 of its size on a refined basis, 40x closer than on a
    coarse one (the Galerkin relation converges with the basis; a wrong sign
    or a missing field term would stay off at order one)."""
    V = lambda x, y: -1.0 / np.sqrt(x * x + y * y + 1.0)
    dV = lambda x, y: x / (x * x + y * y + 1.0) ** 1.5
    errs = []
    for nb in (12, 18):
        bx, by = np.linspace(-7.0, 7.0, nb), np.linspace(-6.0, 6.0, nb - 2)
        m2 = O.assemble_2d(bx, by, 4, 8, V, dVx=dV)
        S2, H2 = dense_2d(m2)
        ev, vec = sl.eigh(H2, S2, subset_by_index=[0, 0])
        dt, ns = 0.01, 100
        E = 0.2 * np.sin(2.0 * dt * np.arange(ns + 1) + 0.3)
        obs, _ = O.propagate_2d(m2, vec[:, 0].astype(np.complex128), E, dt, ns)
        d, a = obs[:, 1], obs[:, 2]
        d2 = (d[2:] - 2.0 * d[1:-1] + d[:-2]) / (dt * dt)
        errs.append(np.abs(d2 - a[1:-1]).max() / np.abs(a).max())
    assert errs[1] < 3e-4 and errs[1] < errs[0] / 20.0, errs
