"""Pins for the oracle's quadrature, B-spline evaluation and Galerkin assembly.

Each check compares the oracle with something other than itself: exactness of
Gauss-Legendre quadrature on polynomials, spline identities (partition of
unity, integral of a B-spline), closed-form element matrices of linear and
cubic B-splines on uniform knots, and SciPy's independent B-spline evaluator.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy.interpolate import BSpline

from oracle import oracle as O
from paper_2608_18472_amd import workloads as W


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 16, 24])
def test_gauss_legendre_exact_on_polynomials(n):
    x, w = O.gauss_legendre(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs((w * x**k).sum() - exact) < 2e-14
    # degree 2n is not integrated exactly (the rule is exactly of degree 2n-1)
    if n <= 10:
        k = 2 * n
        assert abs((w * x**k).sum() - 2.0 / (k + 1)) > 1e-12
    # agrees with NumPy's Golub-Welsch implementation
    xr, wr = leggauss(n)
    assert np.allclose(x, xr, atol=1e-14, rtol=0)
    assert np.allclose(w, wr, atol=1e-14, rtol=0)


def _knots(br, order):
    p = order - 1
    return np.r_[[br[0]] * p, br, [br[-1]] * p]


@pytest.mark.parametrize("order", [2, 3, 4, 6, 8])
def test_bspline_partition_of_unity_and_scipy(order):
    rng = np.random.default_rng(3)
    br = np.sort(np.r_[-3.0, 4.0, rng.uniform(-3, 4, 9)])
    x = np.sort(rng.uniform(-3, 4, 200))
    vals, ders = O.bspline_values(br, order, x)
    assert np.allclose(vals.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(ders.sum(axis=1), 0.0, atol=1e-10)
    t = _knots(br, order)
    ref = BSpline.design_matrix(x, t, order - 1).toarray()
    assert np.abs(vals - ref).max() < 1e-14
    nb = len(t) - order
    dref = np.column_stack([BSpline(t, np.eye(nb)[i], order - 1).derivative()(x) for i in range(nb)])
    assert np.abs(ders - dref).max() < 1e-11 * max(1.0, np.abs(dref).max())


@pytest.mark.parametrize("order", [3, 5, 8])
def test_bspline_integral_closed_form(order):
    """int B_i = (t_{i+k} - t_i) / k for the order-k B-spline B_i."""
    br = np.array([0.0, 0.3, 1.0, 1.1, 2.5, 3.0, 4.2])
    t = _knots(br, order)
    xg, wg = O.quad_points(br, 10)
    vals, _ = O.bspline_values(br, order, xg)
    integ = (vals * wg[:, None]).sum(axis=0)
    nb = len(t) - order
    exact = np.array([(t[i + order] - t[i]) / order for i in range(nb)])
    assert np.allclose(integ, exact, atol=1e-14, rtol=1e-13)


def test_linear_elements_closed_form():
    """Order 2 (hat functions), uniform spacing h: S = h/6 [1 4 1],
    T = (1/(2h)) [-1 2 -1], D_ii = 2h x_i / 3, D_i,i+1 = h (x_i + x_{i+1}) / 12."""
    L, nel = 2.0, 20
    br = W.breaks_uniform(L, nel)
    h = br[1] - br[0]
    m = O.assemble(br, 2, 4)
    N = m["N"]
    assert N == nel - 1 and m["p"] == 1
    xi = br[1:-1]
    assert np.allclose(m["S"][0], 4 * h / 6, atol=1e-15)
    assert np.allclose(m["S"][1, :N - 1], h / 6, atol=1e-15)
    assert np.allclose(m["T"][0], 1.0 / h, atol=1e-13)
    assert np.allclose(m["T"][1, :N - 1], -0.5 / h, atol=1e-13)
    assert np.allclose(m["D"][0], 2 * h * xi / 3, atol=1e-14)
    assert np.allclose(m["D"][1, :N - 1], h * (xi[:-1] + xi[1:]) / 12, atol=1e-14)
    assert np.all(m["S"][1, N - 1:] == 0.0)


def test_cubic_mass_matrix_interior_rows():
    """Uniform cubic B-splines: an interior row of S is h times the order-8
    cardinal B-spline at the integers, [1, 120, 1191, 2416, 1191, 120, 1]/5040."""
    h = 0.25
    br = h * np.arange(41)
    m = O.assemble(br, 4, 6)
    ref = np.array([2416, 1191, 120, 1]) / 5040.0 * h
    i = m["N"] // 2
    assert np.allclose(m["S"][:, i], ref, atol=1e-16, rtol=1e-13)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_row_sums_interior(order):
    """Away from the two boundary spans the dropped B-splines do not overlap a
    row, so sum_j S_ij = int B_i, sum_j T_ij = 0 (constant mass) and
    sum_j D_ij = int x B_i."""
    rng = np.random.default_rng(5)
    br = np.sort(np.r_[-5.0, 6.0, rng.uniform(-5, 6, 30)])
    m = O.assemble(br, order, 10, V=lambda x: np.cos(x), dV=lambda x: -np.sin(x))
    S, T, D = (O.band_to_dense(m[k]) for k in ("S", "T", "D"))
    t = _knots(br, order)
    xq, wq = O.quad_points(br, 10)
    vals, _ = O.bspline_values(br, order, xq)
    p = order - 1
    for i in range(p, m["N"] - p):  # unknown i is B-spline i+1
        gi = i + 1
        assert abs(S[i].sum() - (t[gi + order] - t[gi]) / order) < 1e-13
        assert abs(T[i].sum()) < 1e-10 * np.abs(T[i]).max()
        assert abs(D[i].sum() - (wq * xq * vals[:, gi]).sum()) < 1e-12


def test_assembly_matches_scipy_galerkin():
    """Independent assembly with SciPy's B-spline evaluator and NumPy's
    Gauss-Legendre rule on a graded, position-dependent-mass problem."""
    br = W.breaks_symtann(-10.0, 12.0, 40, 1.5)
    order, nq = 7, 8
    minv = lambda x: 1.0 / (1.0 + 0.3 * np.tanh(x))
    V = lambda x: -1.0 / np.sqrt(x * x + 1.3)
    dV = lambda x: x / (x * x + 1.3) ** 1.5
    m = O.assemble(br, order, nq, minv, V, dV)
    t = _knots(br, order)
    xg, wg = leggauss(nq)
    xs = np.concatenate([(a + b) / 2 + (b - a) / 2 * xg for a, b in zip(br[:-1], br[1:])])
    ws = np.concatenate([(b - a) / 2 * wg for a, b in zip(br[:-1], br[1:])])
    B = BSpline.design_matrix(xs, t, order - 1).toarray()[:, 1:-1]
    nb = len(t) - order
    dB = np.column_stack([BSpline(t, np.eye(nb)[i], order - 1).derivative()(xs) for i in range(nb)])[:, 1:-1]
    ref = {
        "S": (B * ws[:, None]).T @ B,
        "T": 0.5 * (dB * (ws * minv(xs))[:, None]).T @ dB,
        "V": (B * (ws * V(xs))[:, None]).T @ B,
        "D": (B * (ws * xs)[:, None]).T @ B,
        "G": (B * (ws * minv(xs) * dV(xs))[:, None]).T @ B,
        "Mi": (B * (ws * minv(xs))[:, None]).T @ B,
    }
    for k, R in ref.items():
        A = O.band_to_dense(m[k])
        assert np.abs(A - R).max() < 1e-12 * max(1.0, np.abs(R).max()), k
        # the band holds everything: R is zero beyond bandwidth p
        far = np.abs(np.subtract.outer(np.arange(len(R)), np.arange(len(R)))) > order - 1
        assert np.all(R[far] == 0.0)


def test_overlap_spd_and_kinetic_psd():
    m = O.assemble(W.breaks_symexp(30.0, 60, 2.0), 8, 10)
    S = O.band_to_dense(m["S"])
    T = O.band_to_dense(m["T"])
    assert np.linalg.eigvalsh(S).min() > 0
    assert np.linalg.eigvalsh(T).min() > 0  # Dirichlet: T positive definite
