"""GPU three-dimensional tensor-product path against the FP64 oracle.

Reduced anisotropic hydrogen box (13 x 15 x 17 unknowns, cubic splines,
hydrogenic grading on every axis, ragged against the 16 x 4 x 4 and
32 x 4 x 2 tiles): the potential stencil and the operator element by element
(1e-13 relative), the propagation series and final state against the
oracle's Crank-Nicolson run (FP64 1e-10, FP32-refined 1e-8; both drive the
same FP64 residual below 1e-13).  Full size (97^3, the strong-scaling
workload): sampled stencil rows and operator entries against the oracle's
row-by-row definitions, then 100 steps in both precisions checked by
properties that hold at any size (norm conservation, FP32-refined against
FP64 within the 1e-5 dipole bar)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_18472_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_18472_amd import tdsez as T  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def product_state(sd):
    """Product of the 1D ground states of each axis with the 1D potential
    -1/sqrt(x^2 + 1) (oracle eigensolver), as [z][y][x]."""
    vecs = []
    for br in (sd.breaks_x, sd.breaks_y, sd.breaks_z):
        m = O.assemble(br, sd.order, sd.nq, V=lambda x: -1.0 / np.sqrt(x * x + 1.0))
        ev, vec = O.eig_banded(m["H0"], m["S"], 1, -1.5)
        vecs.append(vec[0])
    return np.einsum("z,y,x->zyx", vecs[2], vecs[1], vecs[0]).astype(np.complex128)


def run_gpu_3d(g, sd, psi0, nsteps, prec, tol=1e-13):
    psi = torch.from_numpy(psi0.reshape(-1).copy()).cuda()
    E = torch.from_numpy(np.asarray(sd.E[: nsteps + 1], np.float64).copy()).cuda()
    o = torch.zeros(3 * (nsteps + 1), dtype=torch.float64, device="cuda")
    T.propagate_3d(g, psi, E, sd.dt, nsteps, prec, T.OBS_NORM | T.OBS_DIPOLE, o, tol=tol, maxit=300)
    steps, its, mx, sweeps = T.system3d_stats(g)
    say("3D prec %d: %d steps, %.2f Krylov iterations per step (max %d), %.2f sweeps per step" % (
        prec, steps, its / max(steps, 1), mx, sweeps / max(steps, 1)))
    return o.cpu().numpy().reshape(-1, 3), psi.cpu().numpy()


@pytest.fixture(scope="module")
def small():
    sd = W.hydrogen_3d_small()
    say("3D small case", sd.shape)
    g = T.assemble_workload_3d(sd)
    m3 = O.assemble_3d(sd.breaks_x, sd.breaks_y, sd.breaks_z, sd.order, sd.nq, sd.V)
    assert (g.Nz, g.Ny, g.Nx, g.p) == (m3["Nz"], m3["Ny"], m3["Nx"], m3["p"]) == sd.shape + (3,)
    return sd, g, m3


def test_potential_stencil_matches_oracle(small):
    sd, g, m3 = small
    v = T.get_v3_rows(g, np.arange(g.N))
    ref = m3["V3"]
    err = np.abs(v - ref).max() / np.abs(ref).max()
    say("3D stencil max rel err", err)
    assert err < 1e-13


def test_operator_matches_oracle(small):
    sd, g, m3 = small
    rng = np.random.default_rng(11)
    c = rng.normal(size=g.N) + 1j * rng.normal(size=g.N)
    for a, b, Eb in ((0.7 - 0.2j, 0.3 + 1.1j, 0.37), (1.0, 0.0, 0.0), (0.0, 1.0, -0.8)):
        ref = O.apply_3d(m3, c, a, b, Eb)
        out = torch.zeros(g.N, dtype=torch.complex128, device="cuda")
        T.apply_3d(g, torch.from_numpy(c).cuda(), out, a, b, Eb)
        torch.cuda.synchronize()
        err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
        say("3D operator", a, b, Eb, "max rel err", err)
        assert err < 1e-13


@pytest.mark.parametrize("prec,tol", [(T.FP64, 1e-10), (T.FP32_REFINED, 1e-8)])
def test_small_propagation_matches_oracle(small, prec, tol):
    sd, g, m3 = small
    ns = sd.nsteps
    psi0 = product_state(sd)
    ref, cref = O.propagate_3d(m3, psi0, sd.E, sd.dt, ns, tol=1e-14)
    got, cgot = run_gpu_3d(g, sd, psi0, ns, prec)
    errs = [rel(got[:, k], ref[:, k]) for k in range(2)]
    say("3D small errors", prec, errs, rel(cgot, cref.reshape(-1)))
    assert errs[0] < tol and errs[1] < tol
    assert rel(cgot, cref.reshape(-1)) < tol


@pytest.mark.parametrize("prec", [T.FP64, T.FP32_REFINED])
def test_zero_state_stays_zero(small, prec):
    sd, g, m3 = small
    psi = torch.zeros(g.N, dtype=torch.complex128, device="cuda")
    E = torch.from_numpy(sd.E[:6].copy()).cuda()
    o = torch.zeros(18, dtype=torch.float64, device="cuda")
    T.propagate_3d(g, psi, E, sd.dt, 5, prec, 3, o)
    assert float(psi.abs().max()) == 0.0
    assert float(o.abs().max()) == 0.0


@pytest.mark.parametrize("prec", [T.FP64, T.FP32_REFINED])
def test_exhausted_iteration_budget_latches_enoconv(small, prec):
    sd, g, m3 = small
    psi0 = product_state(sd)
    E = torch.from_numpy(sd.E[:5].copy()).cuda()
    o = torch.zeros(15, dtype=torch.float64, device="cuda")
    psi = torch.from_numpy(psi0.reshape(-1).copy()).cuda()
    with pytest.raises(T.TdsezError) as e:
        T.propagate_3d(g, psi, E, sd.dt, 4, prec, 3, o, tol=1e-14, maxit=1)
    assert e.value.status == 4
    psi = torch.from_numpy(psi0.reshape(-1).copy()).cuda()
    T.propagate_3d(g, psi, E, sd.dt, 4, prec, 3, o, tol=1e-13, maxit=100)
    T.system3d_stats(g)


def test_3d_invalid_arguments(small):
    sd, g, m3 = small
    b = sd.breaks_x
    nq = 4
    n = lambda br: (len(br) - 1) * nq
    Vq = np.zeros(n(b) ** 3)
    with pytest.raises(T.TdsezError) as e:
        T.assemble_3d(b, b, b, 6, nq, Vq)  # order 6: beyond the 3D kernels
    assert e.value.status == 7
    bad = Vq.copy()
    bad[17] = np.nan
    with pytest.raises(T.TdsezError) as e:
        T.assemble_3d(b, b, b, 4, nq, bad)
    assert e.value.status == 1
    short = b[:4]
    with pytest.raises(T.TdsezError) as e:
        T.assemble_3d(short, b, b, 4, nq, np.zeros(n(short) * n(b) ** 2))
    assert e.value.status == 1
    psi = torch.zeros(g.N, dtype=torch.complex128, device="cuda")
    E = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(T.TdsezError) as e:
        T.propagate_3d(g, psi, E, 0.0, 2, T.FP64, 0)
    assert e.value.status == 1
    with pytest.raises(T.TdsezError) as e:
        T.propagate_3d(g, psi, E, 0.01, 2, T.FP64, 4, torch.zeros(9, dtype=torch.float64, device="cuda"))
    assert e.value.status == 1
    with pytest.raises(T.TdsezError) as e:
        T.get_v3_rows(g, [g.N])
    assert e.value.status == 1


def test_full_size_rows_operator_and_100_steps():
    """97^3 hydrogen (912 673 unknowns): sampled stencil rows and operator
    entries against the oracle's definitions, then the 100-step workload in
    both precisions."""
    sd = W.hydrogen_3d()
    g = T.assemble_workload_3d(sd)
    assert (g.Nz, g.Ny, g.Nx) == (97, 97, 97)
    n = g.N
    rng = np.random.default_rng(5)
    centre = (48 * 97 + 48) * 97 + 48
    rows = np.unique(np.r_[0, 1, 96, 97 * 97 - 1, centre, centre - 1, centre + 97 * 97, n - 1,
                           rng.integers(0, n, 16)])
    v = T.get_v3_rows(g, rows)
    ref = O.v3_rows(sd.breaks_x, sd.breaks_y, sd.breaks_z, sd.order, sd.nq, sd.V, rows)
    err = np.abs(v - ref).max() / np.abs(ref).max()
    say("97^3 sampled stencil rows: max rel err", err)
    assert err < 1e-12
    m3ax = {}
    for ax, br in (("x", sd.breaks_x), ("y", sd.breaks_y), ("z", sd.breaks_z)):
        m = O.assemble(br, sd.order, sd.nq)
        m3ax.update({"S" + ax: m["S"], "T" + ax: m["T"], "D" + ax: m["D"], "N" + ax: m["N"]})
    m3ax["p"] = 3
    c = rng.normal(size=n) + 1j * rng.normal(size=n)
    a, b, Eb = 1.0, 0.005j, 0.04
    out = torch.zeros(n, dtype=torch.complex128, device="cuda")
    T.apply_3d(g, torch.from_numpy(c).cuda(), out, a, b, Eb)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[rows]
    refa = O.apply_3d_rows(m3ax, ref, rows, c, a, b, Eb)
    err = np.abs(got - refa).max() / np.abs(refa).max()
    say("97^3 sampled operator entries: max rel err", err)
    assert err < 1e-12
    # the workload: 100 steps of 0.01 from a product state
    psi0 = product_state(sd)
    ns = sd.nsteps
    o64, c64 = run_gpu_3d(g, sd, psi0, ns, T.FP64, tol=1e-12)
    o32, c32 = run_gpu_3d(g, sd, psi0, ns, T.FP32_REFINED, tol=1e-12)
    drift = np.abs(o64[:, 0] / o64[0, 0] - 1.0).max()
    say("97^3: norm drift FP64 %.2e, FP32-refined %.2e; dipole FP32-refined vs FP64 %.2e; state %.2e" % (
        drift, np.abs(o32[:, 0] / o32[0, 0] - 1.0).max(), rel(o32[:, 1], o64[:, 1]), rel(c32, c64)))
    assert drift < 1e-10
    assert np.abs(o32[:, 0] / o32[0, 0] - 1.0).max() < 1e-10
    assert rel(o32[:, 1], o64[:, 1]) < 1e-5
    assert np.abs(o64[-1, 1]) > 1e-6  # the field moved the dipole


def test_ground_state_matches_oracle_dense_pencil(small):
    """Lowest level of the reduced box: the library's shifted inverse
    iteration against the oracle's dense generalised eigensolve of the same
    Kronecker-assembled pencil (LAPACK, the definition)."""
    import scipy.linalg as sl
    sd, g, m3 = small
    D = {k: O.band_to_dense(m3[k]) for k in ("Sx", "Tx", "Sy", "Ty", "Sz", "Tz")}
    S3 = np.kron(D["Sz"], np.kron(D["Sy"], D["Sx"]))
    H3 = (np.kron(D["Sz"], np.kron(D["Sy"], D["Tx"])) + np.kron(D["Sz"], np.kron(D["Ty"], D["Sx"]))
          + np.kron(D["Tz"], np.kron(D["Sy"], D["Sx"])))
    n = g.N
    p = m3["p"]
    for row in range(n):  # the potential from the oracle's stencil rows
        iz, rem = divmod(row, g.Ny * g.Nx)
        iy, ix = divmod(rem, g.Nx)
        for dz in range(-p, p + 1):
            for dy in range(-p, p + 1):
                jz, jy = iz + dz, iy + dy
                if not (0 <= jz < g.Nz and 0 <= jy < g.Ny):
                    continue
                for dx in range(-p, p + 1):
                    jx = ix + dx
                    if 0 <= jx < g.Nx:
                        H3[row, (jz * g.Ny + jy) * g.Nx + jx] += m3["V3"][row, dz + p, dy + p, dx + p]
    ev, vec = sl.eigh(H3, S3, subset_by_index=[0, 0])
    e_ref, x_ref = ev[0], vec[:, 0]
    e, psi = T.ground_state_3d(g, -0.8, tol=1e-13, maxit=80)
    x = psi.cpu().numpy().real
    say("3D ground state: library %.15f oracle %.15f" % (e, e_ref))
    assert abs(e - e_ref) < 1e-12 * abs(e_ref)
    x = x * np.sign(x @ S3 @ x_ref)
    assert np.abs(x - x_ref).max() < 1e-7 * np.abs(x_ref).max()
    assert float(psi.imag.abs().max()) == 0.0


def test_ground_state_full_size():
    """97^3 hydrogen: the lowest level of the grid and an eigen-residual
    check through the operator.  The quadrature of the Coulomb singularity
    (knots on the nucleus) is not exact, so the Galerkin upper bound -1/2
    does not hold strictly; the paper prints -0.499995 for this grid, and the
    workload's unstated knot and quadrature parameters were read so as to
    reproduce it (a reading, so this comparison checks that the reading
    stays in force rather than pinning the method)."""
    sd = W.hydrogen_3d(nsteps=1)
    g = T.assemble_workload_3d(sd)
    e, psi = T.ground_state_3d(g, -0.6, tol=1e-12)
    say("97^3 hydrogen ground state %.9f (printed: -0.499995)" % e)
    assert abs(e - (-0.499995)) < 2e-6
    out = torch.zeros_like(psi)
    T.apply_3d(g, psi, out, -e, 1.0)  # (H - e S) psi
    s_psi = torch.zeros_like(psi)
    T.apply_3d(g, psi, s_psi, 1.0, 0.0)
    torch.cuda.synchronize()
    res = float(out.abs().norm() / s_psi.abs().norm())
    say("eigen-residual |(H - E S) x| / |S x| = %.2e" % res)
    assert res < 1e-5
