"""ctypes front-end of the FP64 CPU oracle (tdsez_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The GPU library never imports this module and
this module never imports the GPU library.

Band convention (same as the C file): a real symmetric banded matrix is its
upper half band, diagonal-major, shape (p+1, N): band[d, i] = M[i, i+d].
Complex vectors are numpy complex128 arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdsez_oracle.c")
_LIB = os.path.join(_HERE, "libtdsez_oracle.so")


def build(force=False):
    """Compile the oracle with plain gcc (no fast-math, no BLAS, no threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        d = ctypes.c_double
        L.orc_gauss_legendre.argtypes = [i, dp, dp]
        L.orc_ndof.argtypes = [i, i]
        L.orc_quad_points.argtypes = [dp, i, i, dp, dp]
        L.orc_bspline_values.argtypes = [dp, i, i, dp, i, dp, dp]
        L.orc_assemble.argtypes = [dp, i, i, i, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_expect.argtypes = [i, i, dp, dp]
        L.orc_expect.restype = d
        L.orc_eig_dense.argtypes = [i, i, dp, dp, dp, dp]
        L.orc_eig_banded.argtypes = [i, i, dp, dp, i, d, d, i, dp, dp]
        L.orc_propagate.argtypes = [i, i, dp, dp, dp, dp, dp, dp, dp, d, i, dp, dp]
        L.orc_adjoint.argtypes = [i, i, dp, dp, dp, dp, dp, dp, dp, d, i, dp, dp, dp]
        L.orc_assemble_v2.argtypes = [dp, i, dp, i, i, i, dp, dp]
        L.orc_assemble_extra.argtypes = [dp, i, i, i, dp, dp, dp, dp, dp, dp, dp]
        L.orc_assemble_v3.argtypes = [dp, i, dp, i, dp, i, i, i, dp, dp]
        L.orc_apply_3d.argtypes = [i, i, i, i, dp, dp, dp, dp, dp, dp, dp, dp, d, d, d, d, d, dp, dp]
        L.orc_velocity.argtypes = [i, i, dp, dp]
        L.orc_velocity.restype = d
        L.orc_ext_columns.argtypes = [i]
        L.orc_propagate_ext.argtypes = [i, i, dp, dp, dp, dp, dp, dp, dp, dp, dp, i, dp, dp, dp, d, i, dp, dp,
                                        dp]
        L.orc_apply_2d.argtypes = [i, i, i, dp, dp, dp, dp, dp, dp, d, d, d, d, d, dp, dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().orc_gauss_legendre(n, _p(x), _p(w)), "gauss_legendre")
    return x, w


def ndof(nbr, order):
    return lib().orc_ndof(nbr, order)


def quad_points(breaks, nq):
    br = _f64(breaks)
    xq = np.zeros((len(br) - 1) * nq)
    wq = np.zeros_like(xq)
    _check(lib().orc_quad_points(_p(br), len(br), nq, _p(xq), _p(wq)), "quad_points")
    return xq, wq


def bspline_values(breaks, order, x):
    br = _f64(breaks)
    x = _f64(x)
    nb = len(br) + order - 2
    vals = np.zeros((len(x), nb))
    ders = np.zeros((len(x), nb))
    _check(lib().orc_bspline_values(_p(br), len(br), order, _p(x), len(x), _p(vals), _p(ders)),
           "bspline_values")
    return vals, ders


def assemble(breaks, order, nq, minv=None, V=None, dV=None, samples=None):
    """Half bands of S, T, V, D, G, Mi.

    minv, V, dV are callables of x (numpy arrays) sampled at the oracle's own
    quadrature points; alternatively `samples` = (minv_q, V_q, dV_q)."""
    br = _f64(breaks)
    N = ndof(len(br), order)
    p = order - 1
    if samples is None:
        xq, _ = quad_points(br, nq)
        minv_q = _f64(minv(xq)) if minv is not None else np.ones_like(xq)
        V_q = _f64(V(xq)) if V is not None else np.zeros_like(xq)
        dV_q = _f64(dV(xq)) if dV is not None else np.zeros_like(xq)
    else:
        minv_q, V_q, dV_q = (_f64(s) for s in samples)
    out = {k: np.zeros((p + 1, N)) for k in ("S", "T", "V", "D", "G", "Mi")}
    _check(lib().orc_assemble(_p(br), len(br), order, nq, _p(minv_q), _p(V_q), _p(dV_q),
                              _p(out["S"]), _p(out["T"]), _p(out["V"]), _p(out["D"]),
                              _p(out["G"]), _p(out["Mi"])), "assemble")
    out["H0"] = out["T"] + out["V"]
    out["N"] = N
    out["p"] = p
    return out


def band_to_dense(band):
    """Dense symmetric matrix from an upper half band (test helper)."""
    p1, N = band.shape
    A = np.zeros((N, N))
    for d in range(p1):
        idx = np.arange(N - d)
        A[idx, idx + d] = band[d, :N - d]
        A[idx + d, idx] = band[d, :N - d]
    return A


def expect(band, c):
    band = _f64(band)
    c = _c128(c)
    p1, N = band.shape
    return lib().orc_expect(N, p1 - 1, _p(band), _p(c.view(np.float64)))


def eig_dense(H, S):
    H = _f64(H)
    S = _f64(S)
    p1, N = S.shape
    ev = np.zeros(N)
    vec = np.zeros((N, N))
    _check(lib().orc_eig_dense(N, p1 - 1, _p(H), _p(S), _p(ev), _p(vec)), "eig_dense")
    return ev, vec


def eig_banded(H, S, nev, sigma, tol=1e-14, maxit=3000):
    H = _f64(H)
    S = _f64(S)
    p1, N = S.shape
    ev = np.zeros(nev)
    vec = np.zeros((nev, N))
    _check(lib().orc_eig_banded(N, p1 - 1, _p(H), _p(S), nev, float(sigma), float(tol), int(maxit),
                                _p(ev), _p(vec)), "eig_banded")
    return ev, vec


def propagate(m, psi0, E, dt, nsteps, with_accel=True):
    """CN propagation of one system; m = dict from assemble().  Returns
    (obs[nsteps+1, 3] = (nu, d, a), psi_final)."""
    N, p = m["N"], m["p"]
    psi0 = _c128(psi0)
    E = _f64(E)
    assert E.shape[0] >= nsteps + 1
    obs = np.zeros((nsteps + 1, 3))
    out = np.zeros(N, dtype=np.complex128)
    G = _f64(m["G"]) if with_accel else None
    Mi = _f64(m["Mi"]) if with_accel else None
    _check(lib().orc_propagate(N, p, _p(_f64(m["S"])), _p(_f64(m["H0"])), _p(_f64(m["D"])), _p(G), _p(Mi),
                               _p(psi0.view(np.float64)), _p(E), float(dt), int(nsteps), _p(obs),
                               _p(out.view(np.float64))), "propagate")
    return obs, out


def adjoint(m, psi0, E, dt, nsteps, dJdobs, with_accel=True):
    """Discrete adjoint: returns (dJ/dE[nsteps+1], dJ/dpsi0)."""
    N, p = m["N"], m["p"]
    psi0 = _c128(psi0)
    E = _f64(E)
    dJdobs = _f64(dJdobs).reshape(nsteps + 1, 3)
    dJdE = np.zeros(nsteps + 1)
    lam0 = np.zeros(N, dtype=np.complex128)
    G = _f64(m["G"]) if with_accel else None
    Mi = _f64(m["Mi"]) if with_accel else None
    _check(lib().orc_adjoint(N, p, _p(_f64(m["S"])), _p(_f64(m["H0"])), _p(_f64(m["D"])), _p(G), _p(Mi),
                             _p(psi0.view(np.float64)), _p(E), float(dt), int(nsteps), _p(dJdobs),
                             _p(dJdE), _p(lam0.view(np.float64))), "adjoint")
    return dJdE, lam0


def assemble_extra(breaks, order, nq, minv=None, eta=None, g=None, h=None):
    """Half bands of the CAP weight W (mask eta), the velocity matrix's real
    antisymmetric part K (Vel = -(i/2) K, upper half band) and the a_Q
    matrix Q, from the samples g = mu mu' and h = mu' mu'' + mu mu''' of
    mu = m^-1 and its derivatives (see orc_assemble_extra).  Each argument is
    a callable of x or None."""
    br = _f64(breaks)
    N = ndof(len(br), order)
    p = order - 1
    xq, _ = quad_points(br, nq)
    smp = [None if f is None else _f64(f(xq)) for f in (minv, eta, g, h)]
    out = {k: np.zeros((p + 1, N)) for k in ("W", "K", "Q")}
    _check(lib().orc_assemble_extra(_p(br), len(br), order, nq, *[_p(a) for a in smp], _p(out["W"]), _p(out["K"]),
                                    _p(out["Q"])), "assemble_extra")
    return out


def velocity(K, c):
    """c^H Vel c with Vel = -(i/2) K (eq. vel_elem)."""
    K = _f64(K)
    c = _c128(c)
    p1, N = K.shape
    return lib().orc_velocity(N, p1 - 1, _p(K), _p(c.view(np.float64)))


EXT_COLUMNS = ("E_kin", "E_pot", "E_int", "E_tot", "minv", "velocity", "a_Q", "W", "auto_re", "auto_im")


def propagate_ext(m, psi0, E, dt, nsteps, W=None, K=None, Q=None, pop=None, with_accel=True):
    """CN propagation with an optional absorber W and the extended series.
    m = dict from assemble(); W, K, Q half bands from assemble_extra (or
    None); pop: (npop, N) real projection states or None.  Returns
    (obs[nsteps+1, 3], ext[nsteps+1, 10 + npop], psi_final)."""
    N, p = m["N"], m["p"]
    psi0 = _c128(psi0)
    E = _f64(E)
    assert E.shape[0] >= nsteps + 1
    npop = 0 if pop is None else int(np.asarray(pop).shape[0])
    popa = None if pop is None else _f64(np.asarray(pop).reshape(npop, N))
    obs = np.zeros((nsteps + 1, 3))
    ext = np.zeros((nsteps + 1, lib().orc_ext_columns(npop)))
    out = np.zeros(N, dtype=np.complex128)
    G = _f64(m["G"]) if with_accel else None
    Mi = _f64(m["Mi"]) if with_accel else None
    opt = [None if a is None else _f64(a) for a in (W, K, Q)]
    _check(lib().orc_propagate_ext(N, p, _p(_f64(m["S"])), _p(_f64(m["T"])), _p(_f64(m["V"])), _p(_f64(m["D"])),
                                   _p(G), _p(Mi), *[_p(a) for a in opt], npop, _p(popa),
                                   _p(psi0.view(np.float64)), _p(E), float(dt), int(nsteps), _p(obs), _p(ext),
                                   _p(out.view(np.float64))), "propagate_ext")
    return obs, ext, out


# --------------------------------------------------------------------------
# Two dimensions (tensor-product basis, constant mass, x-polarised field)
# --------------------------------------------------------------------------
def quad_grid_2d(breaks_x, breaks_y, nq):
    """Tensor grid of the per-axis quadrature points: (X, Y) with shape
    (nqy, nqx) (y slow), matching the V_q layout of orc_assemble_v2."""
    xq, _ = quad_points(breaks_x, nq)
    yq, _ = quad_points(breaks_y, nq)
    return np.meshgrid(xq, yq)


def assemble_2d(breaks_x, breaks_y, order, nq, V, dVx=None):
    """Matrices of the 2D problem: per-axis S, T, D half bands (1D assembly
    with V = 0) and the potential stencil V2 (orc_assemble_v2) for the
    callable V(x, y); with dVx(x, y) also the stencil G2 of dV/dx (the same
    Galerkin integral with the derivative sampled), for the acceleration of
    section IV.A (eq. pdm_acceleration with m = 1: a = -<dV/dx> - E <1>)."""
    bx, by = _f64(breaks_x), _f64(breaks_y)
    mx = assemble(bx, order, nq)
    my = assemble(by, order, nq)
    X, Y = quad_grid_2d(bx, by, nq)
    Nx, Ny, p = mx["N"], my["N"], mx["p"]
    w2 = 2 * p + 1

    def stencil(f):
        out = np.zeros((Ny * Nx, w2, w2))
        _check(lib().orc_assemble_v2(_p(bx), len(bx), _p(by), len(by), order, nq, _p(_f64(f(X, Y))), _p(out)),
               "assemble_v2")
        return out

    m2 = {"Nx": Nx, "Ny": Ny, "p": p, "Sx": mx["S"], "Tx": mx["T"], "Dx": mx["D"], "Sy": my["S"],
          "Ty": my["T"], "V2": stencil(V)}
    if dVx is not None:
        m2["G2"] = stencil(dVx)
    return m2


def stencil_apply_2d(m2, st, c):
    """(M c) for a matrix given as its (2p+1)^2 stencil per row, st[row, dy+p,
    dx+p] = M[row][(iy+dy) Nx + ix+dx] (the V2 / G2 layout), c of shape
    (Ny, Nx) or flat; a plain sum over the offsets of a zero-padded copy."""
    Nx, Ny, p = m2["Nx"], m2["Ny"], m2["p"]
    cc = np.zeros((Ny + 2 * p, Nx + 2 * p), dtype=np.complex128)
    cc[p:p + Ny, p:p + Nx] = np.asarray(c).reshape(Ny, Nx)
    s4 = st.reshape(Ny, Nx, 2 * p + 1, 2 * p + 1)
    out = np.zeros((Ny, Nx), dtype=np.complex128)
    for dy in range(-p, p + 1):
        for dx in range(-p, p + 1):
            out += s4[:, :, dy + p, dx + p] * cc[p + dy:p + dy + Ny, p + dx:p + dx + Nx]
    return out.reshape(-1)


def apply_2d(m2, c, a, b, Ebar, with_V=True):
    """a S2 c + b (T2 + V2 + Ebar D2) c for complex scalars a, b; c complex
    of shape (Ny, Nx) or flat."""
    c = _c128(np.asarray(c).reshape(-1))
    y = np.zeros_like(c)
    _check(lib().orc_apply_2d(m2["Nx"], m2["Ny"], m2["p"], _p(_f64(m2["Sx"])), _p(_f64(m2["Tx"])),
                              _p(_f64(m2["Dx"])), _p(_f64(m2["Sy"])), _p(_f64(m2["Ty"])),
                              _p(_f64(m2["V2"])) if with_V else None, float(np.real(a)), float(np.imag(a)),
                              float(np.real(b)), float(np.imag(b)), float(Ebar), _p(c.view(np.float64)),
                              _p(y.view(np.float64))), "apply_2d")
    return y


def _fdm_factors(m2):
    """Per-axis generalised eigenpairs T Q = S Q Lambda, Q^T S Q = I (LAPACK
    via scipy): the separable part S2 + i a T2 is diagonal in Q_y (x) Q_x."""
    import scipy.linalg as sl
    lx, Qx = sl.eigh(band_to_dense(m2["Tx"]), band_to_dense(m2["Sx"]))
    ly, Qy = sl.eigh(band_to_dense(m2["Ty"]), band_to_dense(m2["Sy"]))
    return lx, Qx, ly, Qy


def cn_solve_2d(m2, rhs, alpha, Ebar, x0=None, fdm=None, tol=1e-14, maxit=500):
    """Solve (S2 + i a H2(Ebar)) x = rhs (section V.B, eq. cn_system in 2D)
    by conjugate-orthogonal CG (A is complex symmetric), preconditioned by
    the exact inverse of the separable part S2 + i a T2 (per-axis
    eigendecompositions); stops at relative residual tol."""
    Nx, Ny = m2["Nx"], m2["Ny"]
    lx, Qx, ly, Qy = fdm if fdm is not None else _fdm_factors(m2)
    den = 1.0 + 1j * alpha * (ly[:, None] + lx[None, :])

    def A(v):
        return apply_2d(m2, v, 1.0, 1j * alpha, Ebar)

    def M(r):
        R = r.reshape(Ny, Nx)
        Z = (Qy.T @ R @ Qx) / den
        return (Qy @ Z @ Qx.T).reshape(-1)

    b = _c128(np.asarray(rhs).reshape(-1))
    x = np.zeros_like(b) if x0 is None else _c128(np.asarray(x0).reshape(-1)).copy()
    r = b - A(x)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    z = M(r)
    pv = z.copy()
    rho = np.sum(r * z)
    for it in range(1, maxit + 1):
        q = A(pv)
        a = rho / np.sum(pv * q)
        x += a * pv
        r -= a * q
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = M(r)
        rho_new = np.sum(r * z)
        pv = z + (rho_new / rho) * pv
        rho = rho_new
    raise OracleError("cn_solve_2d: no convergence to %g in %d iterations" % (tol, maxit))


def propagate_2d(m2, psi0, E, dt, nsteps, tol=1e-14):
    """Crank-Nicolson propagation in 2D (section V.B with Ebar_n =
    (E_n + E_{n+1})/2): returns obs[n] = (nu_n, d_n) = (c^H S2 c, Re c^H D2 c)
    for n = 0..nsteps, and with G2 in m2 (assemble_2d with dVx) a third
    column, the acceleration a_n = -Re c^H G2 c - E_n nu_n (section IV.A,
    constant mass), and the final state (shape (Ny, Nx))."""
    alpha = 0.5 * dt
    c = _c128(np.asarray(psi0).reshape(-1)).copy()
    fdm = _fdm_factors(m2)
    acc = "G2" in m2
    obs = np.zeros((nsteps + 1, 3 if acc else 2))
    for n in range(nsteps + 1):
        Sc = apply_2d(m2, c, 1.0, 0.0, 0.0, with_V=False)
        # D2 c = (T2 + V2 + 1 * D2) c - (T2 + V2) c
        Dc = apply_2d(m2, c, 0.0, 1.0, 1.0) - apply_2d(m2, c, 0.0, 1.0, 0.0)
        obs[n, 0] = np.real(np.vdot(c, Sc))
        obs[n, 1] = np.real(np.vdot(c, Dc))
        if acc:
            obs[n, 2] = -np.real(np.vdot(c, stencil_apply_2d(m2, m2["G2"], c))) - E[n] * obs[n, 0]
        if n == nsteps:
            break
        Eb = 0.5 * (E[n] + E[n + 1])
        rhs = apply_2d(m2, c, 1.0, -1j * alpha, Eb)
        c, _ = cn_solve_2d(m2, rhs, alpha, Eb, x0=c, fdm=fdm, tol=tol)
    return obs, c.reshape(m2["Ny"], m2["Nx"])


# --------------------------------------------------------------------------
# Three dimensions (tensor-product basis, constant mass, x-polarised field)
# --------------------------------------------------------------------------
def assemble_3d(breaks_x, breaks_y, breaks_z, order, nq, V):
    """Matrices of the 3D problem: per-axis S, T, D half bands (1D assembly
    with V = 0) and the potential stencil V3 (orc_assemble_v3) for the
    callable V(x, y, z) sampled on the tensor grid of the per-axis
    quadrature points."""
    bx, by, bz = _f64(breaks_x), _f64(breaks_y), _f64(breaks_z)
    ms = [assemble(b, order, nq) for b in (bx, by, bz)]
    qs = [quad_points(b, nq)[0] for b in (bx, by, bz)]
    Z, Y, X = np.meshgrid(qs[2], qs[1], qs[0], indexing="ij")
    Vq = _f64(V(X, Y, Z))
    Nx, Ny, Nz, p = ms[0]["N"], ms[1]["N"], ms[2]["N"], ms[0]["p"]
    w = 2 * p + 1
    V3 = np.zeros((Nz * Ny * Nx, w, w, w))
    _check(lib().orc_assemble_v3(_p(bx), len(bx), _p(by), len(by), _p(bz), len(bz), order, nq, _p(Vq), _p(V3)),
           "assemble_v3")
    return {"Nx": Nx, "Ny": Ny, "Nz": Nz, "p": p, "Sx": ms[0]["S"], "Tx": ms[0]["T"], "Dx": ms[0]["D"],
            "Sy": ms[1]["S"], "Ty": ms[1]["T"], "Sz": ms[2]["S"], "Tz": ms[2]["T"], "V3": V3}


def v3_rows(breaks_x, breaks_y, breaks_z, order, nq, V, rows):
    """Rows of the 3D potential matrix straight from its definition (section
    II.C, eq. tensor3d with the tensor Gauss rule):
    V3[i][j] = sum over every quadrature point q of w_q V(q) N_i(q) N_j(q),
    restricted to the points where N_i is non-zero.  Returns
    (len(rows), w, w, w) stencils indexed [dz+p][dy+p][dx+p] (zero for a
    neighbour outside the grid), like the rows of assemble_3d's V3."""
    brs = [_f64(b) for b in (breaks_x, breaks_y, breaks_z)]
    p = order - 1
    w = 2 * p + 1
    axes = []
    for br in brs:
        xq, wq = quad_points(br, nq)
        vals, _ = bspline_values(br, order, xq)
        axes.append((xq, wq, vals[:, 1:-1]))  # reduced basis: first and last dropped
    Nx, Ny, Nz = (a[2].shape[1] for a in axes)
    out = np.zeros((len(rows), w, w, w))
    for r, row in enumerate(rows):
        iz, rem = divmod(int(row), Ny * Nx)
        iy, ix = divmod(rem, Nx)
        loc = []
        for (xq, wq, B), i, n in zip(axes, (ix, iy, iz), (Nx, Ny, Nz)):
            sel = np.nonzero(B[:, i])[0]
            j = np.arange(i - p, i + p + 1)
            ok = (j >= 0) & (j < n)
            Bj = np.zeros((len(sel), w))
            Bj[:, ok] = B[np.ix_(sel, j[ok])]
            loc.append((xq[sel], wq[sel] * B[sel, i], Bj))
        (x, ax, Bx), (y, ay, By), (z, az, Bz) = loc
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        Vl = _f64(V(X, Y, Z))
        out[r] = np.einsum("zk,yl,xm,zyx->klm", az[:, None] * Bz, ay[:, None] * By, ax[:, None] * Bx, Vl)
    return out


def apply_3d_rows(m3, v3rows, rows, c, a, b, Ebar):
    """Entries `rows` of a S3 c + b (T3 + V3 + Ebar D3) c from the per-axis
    bands (Kronecker products written out entry by entry) and the given V3
    rows (e.g. from v3_rows); c complex (Nz*Ny*Nx)."""
    Nx, Ny, Nz, p = m3["Nx"], m3["Ny"], m3["Nz"], m3["p"]
    D = {k: band_to_dense(m3[k]) for k in ("Sx", "Tx", "Dx", "Sy", "Ty", "Sz", "Tz")}
    C = _c128(np.asarray(c)).reshape(Nz, Ny, Nx)
    out = np.zeros(len(rows), dtype=np.complex128)
    for r, row in enumerate(rows):
        iz, rem = divmod(int(row), Ny * Nx)
        iy, ix = divmod(rem, Nx)
        js = [np.arange(max(i - p, 0), min(i + p, n - 1) + 1) for i, n in ((iz, Nz), (iy, Ny), (ix, Nx))]
        jz, jy, jx = js
        sz, tz = D["Sz"][iz, jz], D["Tz"][iz, jz]
        sy, ty = D["Sy"][iy, jy], D["Ty"][iy, jy]
        sx, tx, dx = D["Sx"][ix, jx], D["Tx"][ix, jx], D["Dx"][ix, jx]
        blk = C[np.ix_(jz, jy, jx)]
        S3 = np.einsum("k,l,m->klm", sz, sy, sx)
        H3 = (np.einsum("k,l,m->klm", sz, sy, tx + Ebar * dx) + np.einsum("k,l,m->klm", sz, ty, sx)
              + np.einsum("k,l,m->klm", tz, sy, sx))
        V = v3rows[r][np.ix_(jz - iz + p, jy - iy + p, jx - ix + p)]
        out[r] = a * np.sum(S3 * blk) + b * np.sum((H3 + V) * blk)
    return out


def apply_3d(m3, c, a, b, Ebar, with_V=True):
    """a S3 c + b (T3 + V3 + Ebar D3) c for complex scalars a, b."""
    c = _c128(np.asarray(c).reshape(-1))
    y = np.zeros_like(c)
    _check(lib().orc_apply_3d(m3["Nx"], m3["Ny"], m3["Nz"], m3["p"], *[_p(_f64(m3[k])) for k in
                                                                      ("Sx", "Tx", "Dx", "Sy", "Ty", "Sz", "Tz")],
                              _p(_f64(m3["V3"])) if with_V else None, float(np.real(a)), float(np.imag(a)),
                              float(np.real(b)), float(np.imag(b)), float(Ebar), _p(c.view(np.float64)),
                              _p(y.view(np.float64))), "apply_3d")
    return y


def _fdm_factors_3d(m3):
    """Per-axis generalised eigenpairs T Q = S Q Lambda (LAPACK via scipy):
    S3 + i a T3 is diagonal in Qz (x) Qy (x) Qx."""
    import scipy.linalg as sl
    out = []
    for ax in ("x", "y", "z"):
        lam, Q = sl.eigh(band_to_dense(m3["T" + ax]), band_to_dense(m3["S" + ax]))
        out += [lam, Q]
    return out


def cn_solve_3d(m3, rhs, alpha, Ebar, x0=None, fdm=None, tol=1e-14, maxit=500):
    """Solve (S3 + i a H3(Ebar)) x = rhs by COCG preconditioned with the
    exact inverse of the separable part S3 + i a T3 (section V.B, eq.
    cn_system in 3D); stops at relative residual tol."""
    Nx, Ny, Nz = m3["Nx"], m3["Ny"], m3["Nz"]
    lx, Qx, ly, Qy, lz, Qz = fdm if fdm is not None else _fdm_factors_3d(m3)
    den = 1.0 + 1j * alpha * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :])

    def A(v):
        return apply_3d(m3, v, 1.0, 1j * alpha, Ebar)

    def M(r):
        R = r.reshape(Nz, Ny, Nx)
        Z = np.einsum("zc,yb,xa,cba->zyx", Qz.T, Qy.T, Qx.T, R, optimize=True) / den
        return np.einsum("zc,yb,xa,cba->zyx", Qz, Qy, Qx, Z, optimize=True).reshape(-1)

    b = _c128(np.asarray(rhs).reshape(-1))
    x = np.zeros_like(b) if x0 is None else _c128(np.asarray(x0).reshape(-1)).copy()
    r = b - A(x)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    z = M(r)
    pv = z.copy()
    rho = np.sum(r * z)
    for it in range(1, maxit + 1):
        q = A(pv)
        a = rho / np.sum(pv * q)
        x += a * pv
        r -= a * q
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = M(r)
        rho_new = np.sum(r * z)
        pv = z + (rho_new / rho) * pv
        rho = rho_new
    raise OracleError("cn_solve_3d: no convergence to %g in %d iterations" % (tol, maxit))


def propagate_3d(m3, psi0, E, dt, nsteps, tol=1e-14):
    """Crank-Nicolson propagation in 3D (section V.B, Ebar_n = (E_n +
    E_{n+1})/2): obs[n] = (c^H S3 c, Re c^H D3 c) for n = 0..nsteps and the
    final state (shape (Nz, Ny, Nx))."""
    alpha = 0.5 * dt
    c = _c128(np.asarray(psi0).reshape(-1)).copy()
    fdm = _fdm_factors_3d(m3)
    obs = np.zeros((nsteps + 1, 2))
    for n in range(nsteps + 1):
        Sc = apply_3d(m3, c, 1.0, 0.0, 0.0, with_V=False)
        Dc = apply_3d(m3, c, 0.0, 1.0, 1.0) - apply_3d(m3, c, 0.0, 1.0, 0.0)
        obs[n, 0] = np.real(np.vdot(c, Sc))
        obs[n, 1] = np.real(np.vdot(c, Dc))
        if n == nsteps:
            break
        Eb = 0.5 * (E[n] + E[n + 1])
        rhs = apply_3d(m3, c, 1.0, -1j * alpha, Eb)
        c, _ = cn_solve_3d(m3, rhs, alpha, Eb, x0=c, fdm=fdm, tol=tol)
    return obs, c.reshape(m3["Nz"], m3["Ny"], m3["Nx"])
