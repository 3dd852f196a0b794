"""Seeded synthetic inputs: geometries, material profiles, potentials, pulses.

This module defines *problems*, not the method: breakpoint sequences, the
functions m^-1(x), V(x), V'(x) that a caller samples at quadrature points, and
laser-field samples E_n = E(n dt).  It contains none of the discretisation
arithmetic (no quadrature, no B-splines, no matrices, no propagation), so the
GPU library and the CPU oracle can both be fed from it without sharing code.

Units are Hartree atomic units.  The knot gradings are the coordinate maps of
the paper's Table I (section III); the workloads reproduce the shapes of the
paper's examples (soft-Coulomb atoms, the GaAs/AlGaAs double quantum well of
section VII.B, the Quesne position-dependent-mass oscillator of section VII.A,
the driven harmonic oscillator of Appendix A).  Everything is generated from
parameters and seeds; no dataset is read.
"""
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

BOHR_PER_NM = 18.897261246257703  # 1 nm in bohr
EV_PER_HA = 27.211386245988  # 1 Hartree in eV
MEV_PER_HA = 1000.0 * EV_PER_HA


# --------------------------------------------------------------------------
# Knot gradings (Table I, section III).  t_i runs uniformly over [-1, 1].
# --------------------------------------------------------------------------
def _t(nel):
    return -1.0 + 2.0 * np.arange(nel + 1) / nel


def breaks_uniform(L, nel):
    """x_i = -L + 2 i L / N_elem."""
    return -L + 2.0 * L * np.arange(nel + 1) / nel


def breaks_symexp(L, nel, alpha):
    t = _t(nel)
    return np.sign(t) * L * (np.exp(alpha * np.abs(t)) - 1.0) / (np.exp(alpha) - 1.0)


def breaks_symtan(L, nel, alpha):
    a_s = 0.5 * math.pi * alpha / (alpha + 1.0)
    return L * np.tan(a_s * _t(nel)) / math.tan(a_s)


def breaks_symtann(Lmin, Lmax, nel, beta):
    """Clusters knots toward both ends of [Lmin, Lmax]."""
    return Lmin + 0.5 * (Lmax - Lmin) * (1.0 + np.tanh(beta * _t(nel)) / math.tanh(beta))


def breaks_symtanu(Lmin, Lmax, nel, beta):
    """Clusters knots toward the middle of [Lmin, Lmax]."""
    return Lmin + 0.5 * (Lmax - Lmin) * (1.0 + np.arctanh(_t(nel) * math.tanh(beta)) / beta)


def breaks_hydrogenic(r1, nlin, nexp, Lmax):
    """Radial: linear steps r1 up to r_cross = nlin*r1, then exponential to Lmax."""
    rc = nlin * r1
    lin = r1 * np.arange(nlin + 1)
    k = np.arange(1, nexp + 1)
    ex = rc * np.exp(k * math.log(Lmax / rc) / nexp)
    return np.concatenate([lin, ex])


def breaks_hydrogenic_symmetric(r1, nlin, nexp, Lmax):
    """The radial hydrogenic map mirrored about 0 for a symmetric box."""
    r = breaks_hydrogenic(r1, nlin, nexp, Lmax)
    return np.concatenate([-r[::-1], r[1:]])


def breaks_layered(interfaces, nel_total, beta=2.0):
    """Breakpoints with every material interface on a breakpoint.

    `interfaces` = sorted region boundaries x_0 < ... < x_R (box ends
    included).  Spans are shared among regions in proportion to region length
    (the rounding remainder goes to the widest region); inside each region the
    `symtann` map clusters knots toward the region's two ends, i.e. toward the
    interfaces.  No span straddles a jump of m or V."""
    x = np.asarray(interfaces, dtype=float)
    lens = np.diff(x)
    share = lens / lens.sum() * nel_total
    n = np.maximum(np.floor(share).astype(int), 1)
    n[np.argmax(lens)] += nel_total - n.sum()
    out = [np.array([x[0]])]
    for r in range(len(lens)):
        b = breaks_symtann(x[r], x[r + 1], int(n[r]), beta)
        b[0], b[-1] = x[r], x[r + 1]
        out.append(b[1:])
    return np.concatenate(out)


# --------------------------------------------------------------------------
# Pulses.  E(t) is supplied to the propagator as samples E_n = E(n dt).
# --------------------------------------------------------------------------
def sin2_pulse(E0, omega, ncycles, dt, nsteps=None):
    """E(t) = E0 sin^2(pi t / Tp) sin(omega t) on [0, Tp], 0 afterwards,
    Tp = ncycles 2 pi / omega; nsteps defaults to ceil(Tp/dt)."""
    Tp = ncycles * 2.0 * math.pi / omega
    if nsteps is None:
        nsteps = int(math.ceil(Tp / dt - 1e-9))
    t = dt * np.arange(nsteps + 1)
    E = np.where(t <= Tp, E0 * np.sin(math.pi * t / Tp) ** 2 * np.sin(omega * t), 0.0)
    return E, nsteps, Tp


def trapezoid_pulse(E0, omega, ncycles, ramp_cycles, dt, nsteps=None):
    """E(t) = E0 f(t) sin(omega t) on [0, Tp], 0 afterwards, Tp = ncycles
    2 pi / omega, with an envelope f rising linearly over the first
    ramp_cycles cycles, flat, and falling linearly over the last ramp_cycles;
    nsteps defaults to ceil(Tp/dt)."""
    T1 = 2.0 * math.pi / omega
    Tp = ncycles * T1
    Tr = ramp_cycles * T1
    if nsteps is None:
        nsteps = int(math.ceil(Tp / dt - 1e-9))
    t = dt * np.arange(nsteps + 1)
    f = np.clip(np.minimum(t / Tr, (Tp - t) / Tr), 0.0, 1.0)
    return np.where(t <= Tp, E0 * f * np.sin(omega * t), 0.0), nsteps, Tp


def fourier_pulse(theta, Tp, dt, nsteps):
    """E(t; theta) = sum_j theta_j sin(j pi t / Tp) on [0, Tp] (j = 1..len(theta))."""
    t = dt * np.arange(nsteps + 1)
    j = np.arange(1, len(theta) + 1)
    basis = np.sin(np.outer(t, j) * math.pi / Tp) * (t <= Tp)[:, None]
    return basis @ np.asarray(theta, dtype=float), basis


# --------------------------------------------------------------------------
# Problem description.
# --------------------------------------------------------------------------
@dataclass
class System:
    name: str
    breaks: np.ndarray
    order: int
    minv: Callable
    V: Callable
    dV: Callable
    nq: int = 10
    E: Optional[np.ndarray] = None
    dt: float = 0.0
    nsteps: int = 0
    const_mass: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def p(self):
        return self.order - 1

    @property
    def ndof(self):
        return (len(self.breaks) - 1) + self.order - 3

    def sample(self, xq):
        xq = np.asarray(xq, dtype=float)
        return (np.asarray(self.minv(xq), float), np.asarray(self.V(xq), float),
                np.asarray(self.dV(xq), float))


def _ones(x):
    return np.ones_like(x)


def _zeros(x):
    return np.zeros_like(x)


def soft_coulomb(a):
    return (lambda x: -1.0 / np.sqrt(x * x + a)), (lambda x: x / (x * x + a) ** 1.5)


def harmonic(omega=1.0):
    return (lambda x: 0.5 * omega * omega * x * x), (lambda x: omega * omega * x)


# --------------------------------------------------------------------------
# Workloads.
# --------------------------------------------------------------------------
def soft_core_two_centre(R, eps):
    """1D two-centre soft-core potential of H2+ along the molecular axis,
    V(x) = -1/sqrt((x + R/2)^2 + eps) - 1/sqrt((x - R/2)^2 + eps), and dV/dx."""
    def V(x):
        return -1.0 / np.sqrt((x + 0.5 * R) ** 2 + eps) - 1.0 / np.sqrt((x - 0.5 * R) ** 2 + eps)

    def dV(x):
        return (x + 0.5 * R) / ((x + 0.5 * R) ** 2 + eps) ** 1.5 + (x - 0.5 * R) / ((x - 0.5 * R) ** 2 + eps) ** 1.5
    return V, dV


def h2p_1d(nsteps=None, dt=0.05, r1=0.2, nlin=5000):
    """1D H2+ model of the molecular-HHG section: nuclei clamped at R = 2,
    soft-core eps = 1.472, 30 007 degree-7 B-splines on [-4000, 4000] with the
    hydrogenic grading mirrored about 0 (linear steps r1 up to nlin r1, then
    exponential), 6-cycle trapezoidal pulse w = 0.057, 1e14 W/cm^2
    (E0 = 0.0534) with one-cycle linear ramps, dt = 0.05 (13 228 steps)."""
    order = 8
    p = order - 1
    nel = 30007 - p + 2                      # N = nel + p - 2
    nexp = nel // 2 - nlin
    V, dV = soft_core_two_centre(2.0, 1.472)
    E, ns, Tp = trapezoid_pulse(0.0534, 0.057, 6, 1, dt, nsteps)
    return System("h2p-1d", breaks_hydrogenic_symmetric(r1, nlin, nexp, 4000.0), order, _ones, V, dV, 10, E, dt,
                  ns, True, {"R": 2.0, "eps": 1.472, "E0": 0.0534, "omega": 0.057, "Tp": Tp})


def config1(nsteps=None):
    """1D soft-Coulomb atom V = -1/sqrt(x^2+2), order 8, 1000 uniform
    breakpoints on [-200, 200] (N = 1004), sin^2 pulse w = 0.057, E0 = 0.0534,
    4 cycles, dt = 0.05 (8819 steps)."""
    V, dV = soft_coulomb(2.0)
    E, ns, Tp = sin2_pulse(0.0534, 0.057, 4, 0.05, nsteps)
    return System("soft-coulomb-1d", breaks_uniform(200.0, 999), 8, _ones, V, dV, 10, E, 0.05, ns,
                  True, {"E0": 0.0534, "omega": 0.057, "Tp": Tp})


def dqw_profile(wb_nm, lw_nm, mw, mb, V0_ha):
    """Piecewise-constant conduction band and mass of a symmetric double
    quantum well (section VII.B): barrier |x| < wb/2, wells, outer barriers."""
    xb = 0.5 * wb_nm * BOHR_PER_NM
    xw = xb + lw_nm * BOHR_PER_NM

    def well(x):
        ax = np.abs(x)
        return (ax > xb) & (ax < xw)

    minv = lambda x: np.where(well(x), 1.0 / mw, 1.0 / mb)
    V = lambda x: np.where(well(x), 0.0, V0_ha)
    return minv, V, xb, xw


def config2(wb_nm=4.0, N=1500, nsteps=20000, E0=2e-5, outer_nm=30.0, beta=2.0):
    """1D BenDaniel-Duke GaAs/Al0.3Ga0.7As double quantum well: 10 nm wells,
    barrier wb, m* = 0.067 (well) / 0.0919 (barrier), offset 0.23 eV, box
    +-(wb/2 + 10 + outer) nm, order 8, N unknowns with breakpoints on the four
    interfaces; mid-IR sin^2 pulse (0.3 eV photon, 8 cycles)."""
    order = 8
    p = order - 1
    minv, V, xb, xw = dqw_profile(wb_nm, 10.0, 0.067, 0.0919, 0.23 / EV_PER_HA)
    L = xw + outer_nm * BOHR_PER_NM
    nel = N - p + 2
    br = breaks_layered([-L, -xw, -xb, xb, xw, L], nel, beta)
    omega = 0.3 / EV_PER_HA
    Tp = 8 * 2.0 * math.pi / omega
    dt = Tp / nsteps
    E, ns, _ = sin2_pulse(E0, omega, 8, dt, nsteps)
    return System("dqw-bdd-1d", br, order, minv, V, _zeros, 10, E, dt, ns, False,
                  {"wb_nm": wb_nm, "E0": E0, "omega": omega, "Tp": Tp})


def dqw_static_paper(wb_nm=4.0, N=3000, box_nm=40.0, beta=2.0, order=8):
    """The paper's static DQW (section VII.B): 8 nm wells, m_b = 0.092,
    m_w = 0.067, V0 = 233.7 meV, box +-box_nm."""
    p = order - 1
    minv, V, xb, xw = dqw_profile(wb_nm, 8.0, 0.067, 0.092, 0.2337 / EV_PER_HA)
    L = box_nm * BOHR_PER_NM
    nel = N - p + 2
    br = breaks_layered([-L, -xw, -xb, xb, xw, L], nel, beta)
    return System("dqw-static", br, order, minv, V, _zeros, 10, const_mass=False,
                  meta={"wb_nm": wb_nm})


def config3(nsys=1024, seed=0):
    """Batch of soft-Coulomb systems with seeded uneven sizes and pulses:
    per system, in this order, N ~ U{500..4000}, order ~ U{6,7,8},
    E0 = exp(U(ln 0.02, ln 0.1)), omega ~ U(0.03, 0.08); uniform breakpoints
    on [-200, 200] with N - p + 2 spans, 4-cycle sin^2, dt = 0.05."""
    rng = np.random.default_rng(seed)
    V, dV = soft_coulomb(2.0)
    out = []
    for s in range(nsys):
        N = int(rng.integers(500, 4001))
        order = int(rng.integers(6, 9))
        E0 = float(math.exp(rng.uniform(math.log(0.02), math.log(0.1))))
        omega = float(rng.uniform(0.03, 0.08))
        p = order - 1
        E, ns, Tp = sin2_pulse(E0, omega, 4, 0.05)
        out.append(System("batch-%d" % s, breaks_uniform(200.0, N - p + 2), order, _ones, V, dV, 10, E,
                          0.05, ns, True, {"E0": E0, "omega": omega, "Tp": Tp}))
    return out


@dataclass
class System2D:
    """Tensor-product 2D problem with constant mass and an x-polarised field."""
    name: str
    breaks_x: np.ndarray
    breaks_y: np.ndarray
    order: int
    V: Callable  # V(x, y), vectorised
    nq: int = 10
    E: Optional[np.ndarray] = None
    dt: float = 0.0
    nsteps: int = 0
    meta: dict = field(default_factory=dict)
    dVx: Optional[Callable] = None  # dV/dx (x, y), vectorised: the acceleration observable

    @property
    def p(self):
        return self.order - 1

    @property
    def nx(self):
        return len(self.breaks_x) - 1 + self.p - 2

    @property
    def ny(self):
        return len(self.breaks_y) - 1 + self.p - 2


def config4(n=512, nsteps=None, L=120.0, order=6):
    """2D soft-Coulomb atom V = -1/sqrt(x^2 + y^2 + 1): order 6, n unknowns per
    axis on [-L, L]^2 (n - p + 2 uniform spans), x-polarised 4-cycle sin^2
    pulse E0 = 0.05, w = 0.057, dt = 0.05 (8819 steps for the whole pulse)."""
    p = order - 1
    br = breaks_uniform(L, n - p + 2)
    E, ns, Tp = sin2_pulse(0.05, 0.057, 4, 0.05, nsteps)
    return System2D("soft-coulomb-2d", br, br.copy(), order, lambda x, y: -1.0 / np.sqrt(x * x + y * y + 1.0),
                    10, E, 0.05, ns, {"E0": 0.05, "omega": 0.057, "Tp": Tp},
                    lambda x, y: x / (x * x + y * y + 1.0) ** 1.5)


@dataclass
class System3D:
    """Tensor-product 3D problem with constant mass and an x-polarised field."""
    name: str
    breaks_x: np.ndarray
    breaks_y: np.ndarray
    breaks_z: np.ndarray
    order: int
    V: Callable  # V(x, y, z), vectorised
    nq: int = 4
    E: Optional[np.ndarray] = None
    dt: float = 0.0
    nsteps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def p(self):
        return self.order - 1

    @property
    def shape(self):
        """(Nz, Ny, Nx) unknowns."""
        n = lambda b: len(b) - 1 + self.p - 2
        return n(self.breaks_z), n(self.breaks_y), n(self.breaks_x)


def coulomb_3d(x, y, z):
    """Hydrogen, V = -1/r (no regularisation: the quadrature points of
    knots placed on 0 never reach r = 0)."""
    return -1.0 / np.sqrt(x * x + y * y + z * z)


def hydrogen_3d(nsteps=100, dt=0.01, L=25.0, r1=0.125, nlin=24, nexp=24, order=4, nq=6, E0=0.053, omega=0.057):
    """The strong-scaling workload of section VI (Table II): hydrogen on
    cubic B-splines (order 4), the hydrogenic grading mirrored about 0 on
    every axis of [-L, L]^3 (2 (nlin + nexp) spans: 97 unknowns per axis with
    the defaults; linear steps r1 up to nlin r1 = 3, then exponential to L),
    nq Gauss points per span and axis, 100 steps of dt = 0.01 under an
    x-polarised field E(t) = E0 sin(omega t).  The paper does not give r1,
    nlin, nexp or the quadrature; these defaults reproduce its printed
    ground-state energy of the grid (-0.499995) to 1e-6."""
    br = breaks_hydrogenic_symmetric(r1, nlin, nexp, L)
    t = dt * np.arange(nsteps + 1)
    E = E0 * np.sin(omega * t)
    return System3D("hydrogen-3d", br, br.copy(), br.copy(), order, coulomb_3d, nq, E, dt, nsteps,
                    {"E0": E0, "omega": omega, "r1": r1, "nlin": nlin, "nexp": nexp, "L": L})


def hydrogen_3d_small(n=(8, 7, 6), L=(9.0, 8.0, 7.0), nsteps=20, dt=0.05, order=4, nq=4, E0=0.05, omega=0.3):
    """A reduced anisotropic hydrogen box for parity runs: per axis the
    hydrogenic grading mirrored about 0 with n = nlin + nexp spans a side
    (nlin = n // 2, r1 = 0.5), different lengths per axis so that an axis
    mix-up changes the result; a faster field so that the dipole moves."""
    def axis(k, Lk):
        nl = k // 2
        return breaks_hydrogenic_symmetric(0.5, nl, k - nl, Lk)
    t = dt * np.arange(nsteps + 1)
    return System3D("hydrogen-3d-small", axis(n[0], L[0]), axis(n[1], L[1]), axis(n[2], L[2]), order,
                    coulomb_3d, nq, E0 * np.sin(omega * t), dt, nsteps, {"E0": E0, "omega": omega})


def config5(nsys=64, N=1500, nsteps=20000, ntheta=64, seed=1, wb_nm=4.0):
    """Batch for the pulse-gradient workload: config2 double quantum wells
    (all systems share the geometry) driven by Fourier pulses
    E(t) = sum_j theta_j sin(j pi t / Tp), j = 1..ntheta.  theta is the least
    squares fit of the config2 sin^2 pulse, times (1 + 0.1 g) with g standard
    normal from default_rng(seed), drawn per system in order.  Returns
    (systems, thetas, basis); each system's E is its own pulse."""
    base = config2(wb_nm=wb_nm, N=N, nsteps=nsteps)
    Tp = base.meta["Tp"]
    _, basis = fourier_pulse(np.zeros(ntheta), Tp, base.dt, base.nsteps)
    theta0 = np.linalg.lstsq(basis, base.E[: base.nsteps + 1], rcond=None)[0]
    rng = np.random.default_rng(seed)
    systems, thetas = [], []
    for s in range(nsys):
        th = theta0 * (1.0 + 0.1 * rng.standard_normal(ntheta))
        E = basis @ th
        systems.append(System("dqw-grad-%d" % s, base.breaks, base.order, base.minv, base.V, base.dV, base.nq, E,
                              base.dt, base.nsteps, False, dict(base.meta)))
        thetas.append(th)
    return systems, np.array(thetas), basis


def harmonic_yield(d, dt, omega, qmin=15, qmax=35, beta=8.0):
    """J = sum over DFT frequencies w_q in [qmin w, qmax w] of w_q^4 |X(w_q)|^2,
    X(w) = sum_n W_n d_n exp(i w t_n) dt with the apodisation window of
    section IV.A read as a Kaiser window (beta = 8, numpy's convention) over
    the series, and the DFT grid zero-padded to 2^ceil(log2(4 (n+1)))
    points.  d: torch tensor (any device, float64); differentiable."""
    import torch
    n1 = d.shape[-1]
    nfft = 1 << int(math.ceil(math.log2(4 * n1)))
    win = torch.kaiser_window(n1, periodic=False, beta=beta, dtype=d.dtype, device=d.device)
    X = torch.fft.fft(win * d, n=nfft) * dt
    w = 2.0 * math.pi * torch.fft.fftfreq(nfft, d=dt, device=d.device).to(d.dtype)
    sel = (w >= qmin * omega) & (w <= qmax * omega)
    return torch.sum(w[sel] ** 4 * (X[..., sel].abs() ** 2), dim=-1)


def driven_ho(E0=0.1, dt=0.01, tmax=10.0, L=12.0, nel=200, order=8):
    """1D reduction of Appendix A: m = w = 1, E(t) = E0 sin t, from t = 0."""
    V, dV = harmonic(1.0)
    nsteps = int(round(tmax / dt))
    t = dt * np.arange(nsteps + 1)
    return System("driven-ho", breaks_uniform(L, nel), order, _ones, V, dV, 10, E0 * np.sin(t), dt, nsteps,
                  True, {"E0": E0})


def quesne(nel=8000, order=8, a=2.0, omega=1.0, xmax=50.0):
    """Quesne PDM oscillator (section VII.A): M(x) = (1 + x/a)^-1 on
    [-a, xmax], V_code = V_paper/2 with V_paper = a w^2 x^2 / (4 (x + a))
    (the alpha = a^2 w case); exact levels w (n + 1/2) / 2."""
    minv = lambda x: 1.0 + x / a
    V = lambda x: 0.5 * a * omega * omega * x * x / (4.0 * (x + a))
    return System("quesne", np.linspace(-a, xmax, nel + 1), order, minv, V, _zeros, 10, const_mass=False)


# --------------------------------------------------------------------------
# Absorbing boundary layers and smooth position-dependent masses.
# --------------------------------------------------------------------------
MANOLOPOULOS_C = 2.62206


def manolopoulos_cap(x1, L):
    """Mask eta(x) of a Manolopoulos-type transmission-free absorber on the
    layers x1 <= |x| < L (zero for |x| < x1), m = 1:
        eta(x) = (1/2) (2 pi / delta)^2 f(y),  y = c (|x| - x1) / delta,
        f(y) = 4/(c - y)^2 + 4/(c + y)^2 - 8/c^2,  c = 2.62206,
    delta = L - x1.  f(0) = f'(0) = 0 (smooth onset); eta diverges at the box
    edge |x| = L, where the Dirichlet basis functions vanish to order p, so
    the CAP matrix stays finite."""
    c = MANOLOPOULOS_C
    delta = float(L - x1)
    pref = 0.5 * (2.0 * math.pi / delta) ** 2

    def eta(x):
        ax = np.abs(np.asarray(x, dtype=float))
        y = np.clip(c * (ax - x1) / delta, 0.0, c * (1.0 - 1e-14))
        f = 4.0 / (c - y) ** 2 + 4.0 / (c + y) ** 2 - 8.0 / (c * c)
        return np.where(ax > x1, pref * f, 0.0)
    return eta


def config1_cap(nsteps=None, width=50.0):
    """Config 1 with absorbing layers of `width` bohr at both ends of the
    [-200, 200] box (mask manolopoulos_cap(200 - width, 200))."""
    sd = config1(nsteps)
    sd.meta["eta"] = manolopoulos_cap(200.0 - width, 200.0)
    sd.meta["cap_width"] = width
    return sd


def quesne_aq(a=2.0):
    """Samples for the a_Q matrix of the Quesne mass m^-1 = 1 + x/a:
    g = mu mu' = (1 + x/a)/a and h = mu' mu'' + mu mu''' = 0."""
    return (lambda x: (1.0 + x / a) / a), (lambda x: np.zeros_like(x))


def tanh_mass(b=0.3, s=2.0):
    """Smooth position-dependent inverse mass mu(x) = 1 + b tanh(x/s) and the
    a_Q samples g = mu mu', h = mu' mu'' + mu mu''' (closed-form derivatives
    of tanh).  Returns (mu, dmu, g, h)."""
    def mu(x):
        return 1.0 + b * np.tanh(x / s)

    def d1(x):
        u = np.tanh(x / s)
        return (b / s) * (1.0 - u * u)

    def d2(x):
        u = np.tanh(x / s)
        return -(2.0 * b / s ** 2) * u * (1.0 - u * u)

    def d3(x):
        u = np.tanh(x / s)
        return -(2.0 * b / s ** 3) * (1.0 - u * u) * (1.0 - 3.0 * u * u)

    return mu, d1, (lambda x: mu(x) * d1(x)), (lambda x: d1(x) * d2(x) + mu(x) * d3(x))
