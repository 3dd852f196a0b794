"""Pins for the oracle's Crank-Nicolson propagation, observables and adjoint.

Against: LAPACK banded solves on the same matrices, dense brute force on tiny
systems, the exact Cayley phase of a field-free eigenstate, conservation of
the M-norm and of the field-free energy, the closed-form resonantly driven
harmonic oscillator of the paper's Appendix A (reduced to 1D) with its
second-order time convergence, the constant-mass identity a = d'' and central
finite differences of the adjoint gradient.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import oracle as O
from paper_2608_18472_amd import workloads as W


def _small_system(nel=40, order=6, L=15.0):
    V, dV = W.soft_coulomb(1.5)
    m = O.assemble(W.breaks_symtan(L, nel, 0.8), order, 10, lambda x: np.ones_like(x), V, dV)
    return m


def _ground(m):
    ev, vec = O.eig_banded(m["H0"], m["S"], 1, -2.0)
    return ev[0], vec[0].astype(complex)


def _to_lapack_band(A, p):
    N = A.shape[0]
    ab = np.zeros((2 * p + 1, N), dtype=A.dtype)
    for d in range(-p, p + 1):
        diag = np.diagonal(A, d)
        if d >= 0:
            ab[p - d, d:] = diag
        else:
            ab[p - d, :N + d] = diag
    return ab


def test_one_step_matches_lapack_and_dense():
    m = _small_system()
    p, N = m["p"], m["N"]
    rng = np.random.default_rng(11)
    c0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    E = np.array([0.03, 0.05])
    dt = 0.07
    obs, c1 = O.propagate(m, c0, E, dt, 1)
    S, H0, D = (O.band_to_dense(m[k]) for k in ("S", "H0", "D"))
    Hh = H0 + 0.5 * (E[0] + E[1]) * D
    A = S + 0.5j * dt * Hh
    B = S - 0.5j * dt * Hh
    ref = sl.solve_banded((p, p), _to_lapack_band(A, p), B @ c0)
    assert np.abs(c1 - ref).max() < 1e-13 * np.abs(ref).max()
    ref2 = np.linalg.solve(A, B @ c0)
    assert np.abs(c1 - ref2).max() < 1e-13 * np.abs(ref2).max()
    # observables at n = 0 are the plain quadratic forms of c0
    assert abs(obs[0, 0] - np.real(c0.conj() @ S @ c0)) < 1e-12 * abs(obs[0, 0])
    assert abs(obs[0, 1] - np.real(c0.conj() @ D @ c0)) < 1e-12 * np.abs(D).sum()
    G, Mi = O.band_to_dense(m["G"]), O.band_to_dense(m["Mi"])
    a0 = -np.real(c0.conj() @ G @ c0) - E[0] * np.real(c0.conj() @ Mi @ c0)
    assert abs(obs[0, 2] - a0) < 1e-12 * (abs(a0) + 1)


def test_tiny_brute_force_and_expm_second_order():
    """N = 5: dense CN recursion (NumPy) and the exact exponential propagator
    for E = 0; CN differs from expm by O(dt^2) (ratio ~ 4 per halving)."""
    m = O.assemble(W.breaks_uniform(3.0, 4), 4, 8, V=lambda x: 0.3 * x * x)
    N = m["N"]
    assert N == 5
    S, H0 = O.band_to_dense(m["S"]), O.band_to_dense(m["H0"])
    rng = np.random.default_rng(2)
    c0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    T = 2.0
    errs = []
    for ns in (40, 80, 160):
        dt = T / ns
        obs, cT = O.propagate(m, c0, np.zeros(ns + 1), dt, ns, with_accel=False)
        c = c0.copy()
        A = S + 0.5j * dt * H0
        B = S - 0.5j * dt * H0
        for _ in range(ns):
            c = np.linalg.solve(A, B @ c)
        assert np.abs(cT - c).max() < 1e-12 * np.abs(c).max()
        exact = sl.expm(-1j * T * np.linalg.solve(S, H0)) @ c0
        errs.append(np.abs(cT - exact).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_field_free_eigenstate_cayley_phase():
    """c_n = ((1 - i a e)/(1 + i a e))^n c_0 exactly for an eigenpair (e, c_0)."""
    m = _small_system()
    e0, c0 = _ground(m)
    dt, ns = 0.05, 400
    _, cT = O.propagate(m, c0, np.zeros(ns + 1), dt, ns)
    a = 0.5 * dt
    ph = ((1 - 1j * a * e0) / (1 + 1j * a * e0)) ** ns
    assert np.abs(cT - ph * c0).max() < 1e-12
    # the other sign convention (a mistaken i -> -i) is far off
    assert np.abs(cT - np.conj(ph) * c0).max() > 1e-2


def test_norm_and_zero_field_energy_conserved():
    m = _small_system(nel=80, order=8, L=30.0)
    rng = np.random.default_rng(4)
    N = m["N"]
    c0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    c0 /= math.sqrt(np.real(O.expect(m["S"], c0)))
    ns = 5000
    # norm with a strong field on
    E = 0.2 * np.sin(0.3 * 0.05 * np.arange(ns + 1))
    obs, _ = O.propagate(m, c0, E, 0.05, ns)
    assert np.abs(obs[:, 0] - 1.0).max() < 1e-12
    # field-free energy c^H H0 c
    _, cT = O.propagate(m, c0, np.zeros(ns + 1), 0.05, ns)
    e_in = O.expect(m["H0"], c0)
    e_out = O.expect(m["H0"], cT)
    assert abs(e_out - e_in) < 1e-11 * abs(e_in)  # 5000 steps of round-off


def _driven_ho_error(E0, dt, tmax):
    s = W.driven_ho(E0=E0, dt=dt, tmax=tmax)
    m = O.assemble(s.breaks, s.order, s.nq, s.minv, s.V, s.dV)
    ev, vec = O.eig_banded(m["H0"], m["S"], 1, -1.0)
    assert abs(ev[0] - 0.5) < 1e-13
    obs, _ = O.propagate(m, vec[0].astype(complex), s.E, s.dt, s.nsteps)
    t = s.dt * np.arange(s.nsteps + 1)
    x_exact = 0.5 * E0 * (t * np.cos(t) - np.sin(t))
    a_exact = -x_exact - E0 * np.sin(t)  # -<V'> - E for m = w = 1
    return obs, np.abs(obs[:, 1] - x_exact).max(), np.abs(obs[:, 2] - a_exact).max()


def test_driven_harmonic_oscillator_closed_form_and_order():
    """Appendix A, reduced to 1D: <x>(t) = (E0/2)(t cos t - sin t); the
    acceleration observable -<V'> - E(t); both converge as dt^2 (an
    endpoint-field instead of the averaged H^{n+1/2} would give first order,
    a flipped field sign an O(1) error)."""
    E0, tmax = 0.1, 10.0
    errs = []
    for dt in (0.04, 0.02, 0.01):
        obs, ex, ea = _driven_ho_error(E0, dt, tmax)
        assert np.abs(obs[:, 0] - 1.0).max() < 1e-12
        errs.append((ex, ea))
    assert errs[-1][0] < 1e-4 and errs[-1][1] < 1e-4, errs
    for k in (0, 1):
        for e1, e2 in zip(errs[:-1], errs[1:]):
            assert 3.5 < e1[k] / e2[k] < 4.5, errs


def test_acceleration_is_second_derivative_of_dipole():
    """Constant mass: a = d'' (Ehrenfest); check with a centred difference of
    the dipole series on a soft-Coulomb atom in a smooth pulse."""
    m = _small_system(nel=120, order=8, L=40.0)
    e0, c0 = _ground(m)
    E, ns, _ = W.sin2_pulse(0.03, 0.1, 2, 0.01)
    obs, _ = O.propagate(m, c0, E, 0.01, ns)
    d, a = obs[:, 1], obs[:, 2]
    dd = (d[2:] - 2 * d[1:-1] + d[:-2]) / 0.01**2
    assert np.abs(dd - a[1:-1]).max() < 2e-3 * np.abs(a).max()


@pytest.mark.parametrize("with_accel", [True, False])
def test_adjoint_matches_central_differences(with_accel):
    m = _small_system(nel=20, order=5, L=10.0)
    e0, c0 = _ground(m)
    ns, dt = 60, 0.1
    rng = np.random.default_rng(7)
    E = 0.05 * np.sin(0.4 * dt * np.arange(ns + 1)) + 0.01 * rng.normal(size=ns + 1)
    w = rng.normal(size=(ns + 1, 3))
    if not with_accel:
        w[:, 2] = 0.0

    def J(Ev):
        obs, _ = O.propagate(m, c0, Ev, dt, ns, with_accel=with_accel)
        return float((w * obs).sum() + 0.5 * (obs[:, 1] ** 2).sum())

    obs, _ = O.propagate(m, c0, E, dt, ns, with_accel=with_accel)
    dJ = w.copy()
    dJ[:, 1] += obs[:, 1]
    g, _ = O.adjoint(m, c0, E, dt, ns, dJ, with_accel=with_accel)
    h = 1e-6
    for k in list(range(0, ns + 1, 7)) + [ns]:
        e = np.zeros(ns + 1)
        e[k] = h
        fd = (J(E + e) - J(E - e)) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adjoint_initial_state_gradient():
    """lam_0 is the gradient w.r.t. the initial state: dJ = Re(lam_0^H dc0)."""
    m = _small_system(nel=16, order=4, L=8.0)
    N = m["N"]
    rng = np.random.default_rng(9)
    c0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    ns, dt = 30, 0.1
    E = 0.05 * np.sin(0.5 * dt * np.arange(ns + 1))
    w = rng.normal(size=(ns + 1, 3))
    J = lambda c: float((w * O.propagate(m, c, E, dt, ns)[0]).sum())
    _, lam0 = O.adjoint(m, c0, E, dt, ns, w)
    dc = rng.normal(size=N) + 1j * rng.normal(size=N)
    h = 1e-6
    fd = (J(c0 + h * dc) - J(c0 - h * dc)) / (2 * h)
    assert abs(fd - np.real(np.vdot(lam0, dc))) < 1e-6 * max(1.0, abs(fd))
