"""Pins of the oracle's absorber, velocity, a_Q and extended time series.

Each check ties the oracle to something other than itself: the plain
propagation it extends (bit for bit when the extras are off), an exact
discrete identity of the Crank-Nicolson step (norm loss = absorbed flux),
the exact Cayley phase of an eigenstate, conservation laws, closed forms of
the driven harmonic oscillator (Appendix A), the length-velocity relation of
section II, and Ehrenfest's theorem for stationary states (which fixes the
sign and the factors of the a_Q form).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_18472_amd import workloads as W


def small_cap_system(width=15.0, L=40.0, nel=160):
    V, dV = W.soft_coulomb(2.0)
    br = W.breaks_uniform(L, nel)
    m = O.assemble(br, 8, 10, V=V, dV=dV)
    ex = O.assemble_extra(br, 8, 10, eta=W.manolopoulos_cap(L - width, L))
    return br, m, ex


def moving_packet(br, m, k0=1.5, x0=10.0, w=2.0):
    """Coefficients of a Gaussian packet moving toward +x (S-projection of
    exp(-(x-x0)^2/(2w^2) + i k0 x) on the basis), S-normalised."""
    xq, wq = O.quad_points(br, 10)
    vals, _ = O.bspline_values(br, 8, xq)
    vals = vals[:, 1:-1]
    f = np.exp(-0.5 * ((xq - x0) / w) ** 2 + 1j * k0 * xq)
    rhs = vals.T @ (wq * f)
    S = O.band_to_dense(m["S"])
    c = np.linalg.solve(S, rhs)
    return c / math.sqrt(O.expect(m["S"], c))


def test_extras_off_reproduce_plain_propagation_bit_for_bit():
    br, m, ex = small_cap_system()
    c0 = moving_packet(br, m)
    E = 0.05 * np.sin(0.1 * np.arange(31))
    ref, cref = O.propagate(m, c0, E, 0.05, 30)
    for Wb in (None, np.zeros_like(ex["W"])):
        obs, ext, c = O.propagate_ext(m, c0, E, 0.05, 30, W=Wb)
        assert np.array_equal(obs, ref)
        assert np.array_equal(c, cref)


def test_norm_loss_equals_absorbed_flux_each_step():
    """With H = H0 + E D - i W, the CN step gives exactly
    nu_{n+1} - nu_n = -2 dt cbar^H W cbar, cbar = (c_n + c_{n+1})/2."""
    br, m, ex = small_cap_system()
    c = moving_packet(br, m, k0=2.0, x0=20.0)
    E = 0.03 * np.sin(0.2 * np.arange(200))
    dt = 0.05
    lost = 0.0
    for n in range(150):
        obs, ext, c1 = O.propagate_ext(m, c, E[n:n + 2], dt, 1, W=ex["W"])
        cb = 0.5 * (c + c1)
        flux = -2.0 * dt * O.expect(ex["W"], cb)
        assert abs((obs[1, 0] - obs[0, 0]) - flux) <= 1e-13 * max(1.0, abs(flux)) + 1e-15
        lost += -flux
        c = c1
    # the packet reaches the absorber: a visible part of the norm is gone
    assert lost > 1e-3
    assert abs(O.expect(m["S"], c) - (1.0 - lost)) < 1e-12


def test_absorber_matrix_is_positive_semidefinite_and_vanishes_inside():
    br, m, ex = small_cap_system()
    Wd = O.band_to_dense(ex["W"])
    assert np.linalg.eigvalsh(Wd).min() > -1e-12 * np.abs(Wd).max()
    # basis functions supported inside |x| < 25 see no absorber
    N = m["N"]
    inside = [i for i in range(N) if abs(br[min(i + 1, len(br) - 1)]) < 24.0 and abs(br[max(i - 7, 0)]) < 24.0]
    assert np.abs(Wd[np.ix_(inside, inside)]).max() == 0.0


def test_autocorrelation_of_an_eigenstate_is_the_cayley_phase():
    br, m, ex = small_cap_system()
    ev, vec = O.eig_banded(m["H0"], m["S"], 3, -1.0)
    ns, dt = 100, 0.05
    obs, ext, _ = O.propagate_ext(m, vec[1], np.zeros(ns + 1), dt, ns, pop=vec)
    a = 0.5 * dt
    n = np.arange(ns + 1)
    ph = ((1 - 1j * a * ev[1]) / (1 + 1j * a * ev[1])) ** n
    assert np.abs(ext[:, 8] + 1j * ext[:, 9] - ph).max() < 1e-12
    # populations: all in state 1
    assert np.abs(ext[:, 11] - 1.0).max() < 1e-12
    assert np.abs(ext[:, 10]).max() < 1e-20 and np.abs(ext[:, 12]).max() < 1e-20
    # the mistaken sign (e^{+i eps t}) is far off
    assert np.abs(ext[:, 8] + 1j * ext[:, 9] - np.conj(ph)).max() > 0.1


def test_field_free_energy_is_conserved_and_splits_into_kinetic_and_potential():
    br, m, ex = small_cap_system()
    c0 = moving_packet(br, m, k0=0.7, x0=0.0)
    ns = 400
    obs, ext, _ = O.propagate_ext(m, c0, np.zeros(ns + 1), 0.05, ns)
    H0 = O.expect(m["H0"], c0)
    assert abs(ext[0, 3] - H0) < 1e-13 * abs(H0)
    assert np.abs(ext[:, 3] - ext[0, 3]).max() < 1e-12 * abs(H0)
    assert np.abs(ext[:, 2]).max() == 0.0
    # kinetic and potential parts exchange energy while the total stays put
    assert np.ptp(ext[:, 0]) > 1e-3
    assert np.abs(ext[:, 4] - obs[:, 0]).max() < 1e-13  # <m^-1> = norm for m = 1


def test_populations_are_complete_on_a_tiny_basis():
    br = np.linspace(-4.0, 4.0, 6)
    m = O.assemble(br, 4, 8, V=lambda x: 0.5 * x * x, dV=lambda x: x)
    N = m["N"]
    ev, vec = O.eig_dense(m["H0"], m["S"])
    rng = np.random.default_rng(3)
    c0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    E = 0.3 * np.sin(0.5 * np.arange(21))
    obs, ext, _ = O.propagate_ext(m, c0, E, 0.1, 20, pop=vec)  # rows are the eigenvectors
    assert np.abs(ext[:, 10:].sum(axis=1) - obs[:, 0]).max() < 1e-12 * obs[0, 0]


def test_velocity_of_the_driven_oscillator_matches_the_closed_form():
    """Appendix A (1D): m = w = 1, E = E0 sin t from the ground state gives
    <x> = (E0/2)(t cos t - sin t), hence <v> = -(E0/2) t sin t.  CN has a
    second-order error in dt: halving dt divides it by about four."""
    errs = []
    for dt in (0.02, 0.01):
        sd = W.driven_ho(E0=0.1, dt=dt, tmax=6.0)
        m = O.assemble(sd.breaks, sd.order, sd.nq, None, sd.V, sd.dV)
        ex = O.assemble_extra(sd.breaks, sd.order, sd.nq)
        ev, vec = O.eig_banded(m["H0"], m["S"], 1, -0.1)
        obs, ext, _ = O.propagate_ext(m, vec[0], sd.E, sd.dt, sd.nsteps, K=ex["K"])
        t = sd.dt * np.arange(sd.nsteps + 1)
        errs.append(np.abs(ext[:, 5] - (-0.05 * t * np.sin(t))).max())
    assert errs[0] < 2e-4
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def test_velocity_matrix_obeys_the_length_velocity_relation():
    """Heisenberg's relation v = i [H, x] gives v_mn = i (eps_m - eps_n) d_mn
    for eigenstates, which the matrix of eq. vel_elem obeys; the relation as
    printed in section IV.B has the opposite sign, which is inconsistent with
    that element formula (the element formula is taken as the definition).
    For the harmonic oscillator <0|v|1> has modulus 1/sqrt(2)."""
    sd = W.driven_ho(E0=0.0)
    m = O.assemble(sd.breaks, sd.order, sd.nq, None, sd.V, sd.dV)
    ex = O.assemble_extra(sd.breaks, sd.order, sd.nq)
    ev, vec = O.eig_banded(m["H0"], m["S"], 5, -0.1)
    K = O.band_to_dense(ex["K"])
    K = np.triu(K) - np.triu(K).T  # antisymmetric from the upper half band
    Vel = -0.5j * K
    D = O.band_to_dense(m["D"])
    for a in range(5):
        for b in range(5):
            vmn = vec[a] @ Vel @ vec[b]
            dmn = vec[a] @ D @ vec[b]
            assert abs(vmn - 1j * (ev[a] - ev[b]) * dmn) < 1e-9
    assert abs(abs(vec[0] @ Vel @ vec[1]) - 1.0 / math.sqrt(2.0)) < 1e-9
    # orc_velocity agrees with the dense form
    c = vec[0] + 0.3j * vec[1]
    assert abs(O.velocity(ex["K"], c) - np.real(np.conj(c) @ Vel @ c)) < 1e-13


@pytest.mark.parametrize("which", ["quesne", "tanh-mass"])
def test_aQ_closes_ehrenfest_for_stationary_states(which):
    """For an eigenstate d<v>/dt = 0, so a_Q = <m^-1 V'> (eq.
    pdm_acceleration with E = 0).  Checked on the Quesne mass (linear m^-1,
    h = 0) and on a tanh mass with a harmonic potential (all terms of the
    a_Q form non-zero).  A wrong factor or sign in either term fails."""
    if which == "quesne":
        q = W.quesne(nel=2000)
        br, order = q.breaks, q.order
        mu, V = q.minv, q.V
        a = 2.0
        dV = lambda x: 0.5 * a * x * (x + 2 * a) / (4.0 * (x + a) ** 2)
        g, h = W.quesne_aq(a)
        shift = -0.01
    else:
        br, order = W.breaks_uniform(10.0, 400), 8
        mu, dmu, g, h = W.tanh_mass(0.3, 1.5)
        V, dV = W.harmonic(1.0)
        shift = -0.1
    m = O.assemble(br, order, 10, mu, V, dV)
    ex = O.assemble_extra(br, order, 10, minv=mu, g=g, h=h)
    ev, vec = O.eig_banded(m["H0"], m["S"], 4, shift)
    for k in range(4):
        force = O.expect(m["G"], vec[k])
        aq = O.expect(ex["Q"], vec[k])
        assert abs(aq - force) < 1e-8 * max(1.0, abs(force)), (k, aq, force)
    # the half-weighted derivative term alone would not balance
    ex2 = O.assemble_extra(br, order, 10, minv=mu, g=g)
    if which == "tanh-mass":
        assert abs(O.expect(ex2["Q"], vec[0]) - O.expect(m["G"], vec[0])) > 1e-4


def test_aQ_vanishes_for_constant_mass_and_is_added_to_the_acceleration():
    br, m, ex = small_cap_system()
    ex2 = O.assemble_extra(br, 8, 10, g=lambda x: 0.0 * x + 0.2, h=lambda x: 0.1 + 0.0 * x)
    c0 = moving_packet(br, m, k0=0.5)
    E = 0.02 * np.sin(0.3 * np.arange(11))
    o1, e1, _ = O.propagate_ext(m, c0, E, 0.05, 10)
    o2, e2, _ = O.propagate_ext(m, c0, E, 0.05, 10, Q=ex2["Q"])
    assert np.abs(e1[:, 6]).max() == 0.0
    assert np.abs(o2[:, 2] - (o1[:, 2] + e2[:, 6])).max() < 1e-14
    assert np.abs(e2[:, 6]).max() > 1e-3
