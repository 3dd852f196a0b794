"""Python binding of libtdsez (include/tdsez.h): argument marshalling only.

Every numerical step runs in the HIP library; PyTorch provides device memory
and streams.  The binding raises TdsezError when the library is missing or a
call fails -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdsez.so")

TDSEZ_OK = 0
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOCONV", 5: "ENONFINITE",
                6: "ENORMDRIFT", 7: "EUNSUPPORTED"}
FP64 = 0
FP32_REFINED = 1
OBS_NORM, OBS_DIPOLE, OBS_ACCEL = 1, 2, 4
OBS_ALL = 7
EXT_SERIES = 1
EXT_COLUMNS = ("E_kin", "E_pot", "E_int", "E_tot", "minv", "velocity", "a_Q", "W", "auto_re", "auto_im")
BAND = {"S": 0, "T": 1, "V": 2, "D": 3, "G": 4, "Mi": 5, "H0": 6, "K": 7, "W": 8, "Q": 9}
PROFILE_COLUMNS = 10


class TdsezError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("tdsez %s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_lib = None


def lib():
    """Load libtdsez.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TdsezError(-1, "libtdsez.so not found at %s; build it with __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip, lp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), \
        ctypes.POINTER(ctypes.c_long)
    i, d, u = ctypes.c_int, ctypes.c_double, ctypes.c_uint
    L.tdsez_last_error.restype = ctypes.c_char_p
    L.tdsez_version.restype = i
    sigs = {
        "tdsez_gauss_legendre": [i, dp, dp],
        "tdsez_quad_points": [dp, i, i, dp],
        "tdsez_assemble": [dp, i, i, i, dp, dp, dp, ctypes.POINTER(vp)],
        "tdsez_system_size": [vp, ip, ip],
        "tdsez_get_band": [vp, i, dp],
        "tdsez_ground_state": [vp, i, d, d, i, dp, dp],
        "tdsez_batch_create": [ctypes.POINTER(vp), i, ctypes.POINTER(vp)],
        "tdsez_ground_state_batched": [vp, d, d, i, dp, vp, lp],
        "tdsez_batch_set": [vp, ctypes.c_char_p, d],
        "tdsez_propagate_batched": [vp, vp, lp, vp, lp, dp, ip, i, u, vp, lp, vp],
        "tdsez_propagate": [vp, vp, vp, d, i, i, u, vp, vp],
        "tdsez_propagate_batched_ext": [vp, vp, lp, vp, lp, dp, ip, i, u, vp, lp, u, vp, lp, vp],
        "tdsez_propagate_ext": [vp, vp, vp, d, i, i, u, vp, u, vp, vp],
        "tdsez_propagate_noalloc": [vp, vp, vp, d, i, i, u, vp, vp, vp],
        "tdsez_set_cap": [vp, dp],
        "tdsez_set_aq": [vp, dp, dp],
        "tdsez_set_projectors": [vp, i, dp],
        "tdsez_ext_columns": [vp, ip],
        "tdsez_adjoint_batched": [vp, vp, lp, vp, lp, dp, ip, i, u, vp, lp, vp, vp, i, vp],
        "tdsez_assemble_2d": [dp, i, dp, i, i, i, dp, dp, ctypes.POINTER(vp)],
        "tdsez_system2d_size": [vp, ip, ip, ip],
        "tdsez_get_v2": [vp, dp],
        "tdsez_propagate_2d": [vp, vp, vp, d, i, i, u, vp, d, i, vp],
        "tdsez_system2d_stats": [vp, lp, lp, ip, lp],
        "tdsez_assemble_3d": [dp, i, dp, i, dp, i, i, i, dp, ctypes.POINTER(vp)],
        "tdsez_system3d_size": [vp, ip, ip, ip, ip],
        "tdsez_get_v3_rows": [vp, lp, i, dp],
        "tdsez_apply_3d": [vp, vp, vp, d, d, d, d, d, vp],
        "tdsez_propagate_3d": [vp, vp, vp, d, i, i, u, vp, d, i, vp],
        "tdsez_system3d_stats": [vp, lp, lp, ip, lp],
        "tdsez_time_apply_3d": [vp, i, i, vp, dp],
        "tdsez_ground_state_3d": [vp, d, d, i, vp, dp],
        "tdsez_time_apply_2d": [vp, i, i, vp, dp],
        "tdsez_batch_status": [vp, vp, ip, ip],
        "tdsez_batch_profile": [vp, vp, dp],
        "tdsez_autotune": [vp, i, d],
        "tdsez_batch_chunks": [vp, ip],
        "tdsez_batch_split": [vp, ip, ctypes.c_int],
        "tdsez_batch_two_wave": [vp, ip],
        "tdsez_batch_waves": [vp, ip],
        "tdsez_system_status": [vp, vp, ip],
        "tdsez_system_set": [vp, ctypes.c_char_p, d],
        "tdsez_system_workgroups": [vp, ip, ip],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i
    L.tdsez_batch_destroy.argtypes = [vp]
    L.tdsez_batch_destroy.restype = None
    L.tdsez_system_destroy.argtypes = [vp]
    L.tdsez_system_destroy.restype = None
    L.tdsez_system2d_destroy.argtypes = [vp]
    L.tdsez_system2d_destroy.restype = None
    L.tdsez_system3d_destroy.argtypes = [vp]
    L.tdsez_system3d_destroy.restype = None
    _lib = L
    return L


def _check(st):
    if st != TDSEZ_OK:
        raise TdsezError(st, lib().tdsez_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


def version():
    return lib().tdsez_version()


def gauss_legendre(nq):
    x = np.zeros(nq)
    w = np.zeros(nq)
    _check(lib().tdsez_gauss_legendre(nq, _dptr(x), _dptr(w)))
    return x, w


def quad_points(breaks, nq):
    br = _f64(breaks)
    x = np.zeros((len(br) - 1) * nq)
    _check(lib().tdsez_quad_points(_dptr(br), len(br), nq, _dptr(x)))
    return x


class System:
    """An assembled 1D problem (owns FP64 device bands)."""

    def __init__(self, handle):
        self.handle = handle
        N = ctypes.c_int()
        p = ctypes.c_int()
        _check(lib().tdsez_system_size(handle, ctypes.byref(N), ctypes.byref(p)))
        self.N, self.p = N.value, p.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tdsez_system_destroy(self.handle)
            self.handle = None


def assemble(breaks, order, nq, minv_q=None, V_q=None, dV_q=None):
    br = _f64(breaks)
    arrs = [None if a is None else _f64(a) for a in (minv_q, V_q, dV_q)]
    h = ctypes.c_void_p()
    _check(lib().tdsez_assemble(_dptr(br), len(br), order, nq,
                                *[None if a is None else _dptr(a) for a in arrs], ctypes.byref(h)))
    return System(h)


def assemble_workload(sysdef):
    """Assemble a workloads.System: sample its m^-1, V, V' at the library's
    own quadrature points; an absorber mask meta["eta"] and a_Q samples
    meta["aq"] = (g, h) (callables) are set as well."""
    xq = quad_points(sysdef.breaks, sysdef.nq)
    minv, V, dV = sysdef.sample(xq)
    g = assemble(sysdef.breaks, sysdef.order, sysdef.nq, None if sysdef.const_mass else minv, V, dV)
    meta = getattr(sysdef, "meta", None) or {}
    if meta.get("eta") is not None:
        set_cap(g, meta["eta"](xq))
    if meta.get("aq") is not None:
        fg, fh = meta["aq"]
        set_aq(g, None if fg is None else fg(xq), None if fh is None else fh(xq))
    return g


def set_cap(sys, eta_q):
    """Absorbing potential from the mask samples at the quadrature points
    (None removes it)."""
    a = None if eta_q is None else _f64(eta_q)
    _check(lib().tdsez_set_cap(sys.handle, None if a is None else _dptr(a)))


def set_aq(sys, g_q, h_q):
    """a_Q form from samples of g = mu mu_1 and h = mu_1 mu_2 + mu mu_3."""
    a = None if g_q is None else _f64(g_q)
    b = None if h_q is None else _f64(h_q)
    _check(lib().tdsez_set_aq(sys.handle, None if a is None else _dptr(a), None if b is None else _dptr(b)))


def set_projectors(sys, phi):
    """Projection states of the population series: (npop, N) real array, or
    None / empty to remove them."""
    if phi is None or len(phi) == 0:
        _check(lib().tdsez_set_projectors(sys.handle, 0, None))
        return
    a = _f64(np.asarray(phi).reshape(len(phi), sys.N))
    _check(lib().tdsez_set_projectors(sys.handle, a.shape[0], _dptr(a)))


def ext_columns(sys):
    n = ctypes.c_int()
    _check(lib().tdsez_ext_columns(sys.handle, ctypes.byref(n)))
    return n.value


def system_size(sys):
    return sys.N, sys.p


def get_band(sys, which):
    out = np.zeros((sys.p + 1) * sys.N)
    _check(lib().tdsez_get_band(sys.handle, BAND[which] if isinstance(which, str) else which, _dptr(out)))
    return out.reshape(sys.p + 1, sys.N)


def ground_state(sys, nev=1, sigma=None, tol=1e-13, maxit=5000):
    eps = np.zeros(nev)
    vec = np.zeros(nev * sys.N)
    _check(lib().tdsez_ground_state(sys.handle, nev, 1e301 if sigma is None else float(sigma), tol, maxit,
                                    _dptr(eps), _dptr(vec)))
    return eps, vec.reshape(nev, sys.N)


class Batch:
    def __init__(self, handle, systems):
        self.handle = handle
        self.systems = list(systems)  # keep the systems alive

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tdsez_batch_destroy(self.handle)
            self.handle = None


def batch_create(systems):
    arr = (ctypes.c_void_p * len(systems))(*[s.handle for s in systems])
    h = ctypes.c_void_p()
    _check(lib().tdsez_batch_create(arr, len(systems), ctypes.byref(h)))
    return Batch(h, systems)


def ground_state_batched(batch, psi_packed, psi_off, sigma=None, tol=1e-13, maxit=20000):
    """Ground states of every system, written into the device complex128
    buffer psi_packed at the host offsets psi_off; returns the energies."""
    import torch
    _check_dev(psi_packed, torch.complex128)
    eps = np.zeros(len(batch.systems))
    po, pp = _longs(psi_off)
    _check(lib().tdsez_ground_state_batched(batch.handle, 1e301 if sigma is None else float(sigma), tol, maxit,
                                            _dptr(eps), ctypes.c_void_p(psi_packed.data_ptr()), pp))
    return eps


def batch_set(batch, key, value):
    _check(lib().tdsez_batch_set(batch.handle, key.encode(), float(value)))


def _longs(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def _check_dev(t, dtype):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TdsezError(1, "expected a contiguous CUDA tensor of dtype %s" % dtype)


def propagate_batched(batch, psi_packed, psi_off, E_packed, E_off, dt, nsteps, prec=FP64, obs=OBS_ALL,
                      obs_packed=None, obs_off=None, stream=None, ext=0, ext_packed=None, ext_off=None):
    """psi_packed: torch complex128 (device, in/out); E_packed: torch float64
    (device); obs_packed: torch float64 (device) or None; with ext =
    EXT_SERIES the extended series go to ext_packed (device float64) at the
    host offsets ext_off.  Offsets, dt and nsteps are host sequences."""
    import torch
    _check_dev(psi_packed, torch.complex128)
    _check_dev(E_packed, torch.float64)
    n = len(batch.systems)
    po, pp = _longs(psi_off)
    eo, ep = _longs(E_off)
    dtv = _f64(dt)
    ns = np.ascontiguousarray(nsteps, dtype=np.int32)
    if len(po) != n or len(eo) != n or len(dtv) != n or len(ns) != n:
        raise TdsezError(1, "per-system arrays must have one entry per system")
    if obs:
        _check_dev(obs_packed, torch.float64)
        oo, op_ = _longs(obs_off)
        optr = ctypes.c_void_p(obs_packed.data_ptr())
    else:
        oo, op_ = _longs(np.zeros(n))
        optr = None
    if ext:
        _check_dev(ext_packed, torch.float64)
        xo, xp = _longs(ext_off)
        if len(xo) != n:
            raise TdsezError(1, "per-system arrays must have one entry per system")
        xptr = ctypes.c_void_p(ext_packed.data_ptr())
    else:
        xo, xp = _longs(np.zeros(n))
        xptr = None
    _check(lib().tdsez_propagate_batched_ext(batch.handle, ctypes.c_void_p(psi_packed.data_ptr()), pp,
                                             ctypes.c_void_p(E_packed.data_ptr()), ep, _dptr(dtv),
                                             ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(prec), int(obs),
                                             optr, op_, int(ext), xptr, xp, _stream_handle(stream)))


def adjoint_batched(batch, psi0_packed, psi_off, E_packed, E_off, dt, nsteps, obs, dJdobs_packed, obs_off,
                    dJdE_packed, dJdpsi0_packed=None, ckpt_stride=0, prec=FP64, stream=None):
    """Discrete-adjoint gradient of J(observable series): fills dJdE_packed
    (device float64, E layout) and optionally dJdpsi0_packed (device
    complex128, psi layout) from dJdobs_packed (device float64, obs layout)."""
    import torch
    _check_dev(psi0_packed, torch.complex128)
    _check_dev(E_packed, torch.float64)
    _check_dev(dJdobs_packed, torch.float64)
    _check_dev(dJdE_packed, torch.float64)
    if dJdpsi0_packed is not None:
        _check_dev(dJdpsi0_packed, torch.complex128)
    n = len(batch.systems)
    po, pp = _longs(psi_off)
    eo, ep = _longs(E_off)
    oo, op_ = _longs(obs_off)
    dtv = _f64(dt)
    ns = np.ascontiguousarray(nsteps, dtype=np.int32)
    if len(po) != n or len(eo) != n or len(oo) != n or len(dtv) != n or len(ns) != n:
        raise TdsezError(1, "per-system arrays must have one entry per system")
    _check(lib().tdsez_adjoint_batched(batch.handle, ctypes.c_void_p(psi0_packed.data_ptr()), pp,
                                       ctypes.c_void_p(E_packed.data_ptr()), ep, _dptr(dtv),
                                       ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(prec), int(obs),
                                       ctypes.c_void_p(dJdobs_packed.data_ptr()), op_,
                                       ctypes.c_void_p(dJdE_packed.data_ptr()),
                                       None if dJdpsi0_packed is None else ctypes.c_void_p(dJdpsi0_packed.data_ptr()),
                                       int(ckpt_stride), _stream_handle(stream)))


def _series_function():
    import torch

    class ObservableSeries(torch.autograd.Function):
        """E samples (device float64, packed) -> observable series (device
        float64, packed [n*3 + (nu, d, a)]) of a batch propagated from fixed
        initial states; backward runs tdsez_adjoint_batched (FP64)."""

        @staticmethod
        def forward(ctx, E_packed, batch, psi0_packed, psi_off, E_off, dt, nsteps, obs_off, obs, prec, ckpt_stride):
            psi = psi0_packed.clone()
            total = max(int(o) + 3 * (int(k) + 1) for o, k in zip(obs_off, nsteps))
            series = torch.zeros(total, dtype=torch.float64, device=E_packed.device)
            propagate_batched(batch, psi, psi_off, E_packed.detach().contiguous(), E_off, dt, nsteps, prec, obs,
                              series, obs_off)
            batch_status(batch)
            ctx.save_for_backward(E_packed.detach(), psi0_packed)
            ctx.args = (batch, psi_off, E_off, dt, nsteps, obs_off, obs, ckpt_stride)
            return series

        @staticmethod
        def backward(ctx, grad_series):
            E_packed, psi0_packed = ctx.saved_tensors
            batch, psi_off, E_off, dt, nsteps, obs_off, obs, ckpt_stride = ctx.args
            dJdE = torch.zeros_like(E_packed)
            adjoint_batched(batch, psi0_packed, psi_off, E_packed.contiguous(), E_off, dt, nsteps, obs,
                            grad_series.contiguous(), obs_off, dJdE, None, ckpt_stride, FP64)
            batch_status(batch)
            return dJdE, None, None, None, None, None, None, None, None, None, None

    return ObservableSeries


_OBS_FN = None


def observable_series(E_packed, batch, psi0_packed, psi_off, E_off, dt, nsteps, obs_off, obs=OBS_ALL, prec=FP64,
                      ckpt_stride=0):
    """Differentiable propagation: returns the packed observable series as a
    torch tensor whose gradient with respect to E_packed comes from the
    discrete adjoint (tdsez_adjoint_batched)."""
    global _OBS_FN
    if _OBS_FN is None:
        _OBS_FN = _series_function()
    return _OBS_FN.apply(E_packed, batch, psi0_packed, psi_off, E_off, dt, nsteps, obs_off, obs, prec, ckpt_stride)


def propagate(sys, psi, E, dt, nsteps, prec=FP64, obs=OBS_ALL, obs_out=None, stream=None, ext=0, ext_out=None):
    """Single-system propagation; with ext = EXT_SERIES the extended series
    go to ext_out (device float64, (nsteps+1) * ext_columns(sys))."""
    import torch
    _check_dev(psi, torch.complex128)
    _check_dev(E, torch.float64)
    if obs:
        _check_dev(obs_out, torch.float64)
    if ext:
        _check_dev(ext_out, torch.float64)
    _check(lib().tdsez_propagate_ext(sys.handle, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                     float(dt), int(nsteps), int(prec), int(obs),
                                     ctypes.c_void_p(obs_out.data_ptr()) if obs else None, int(ext),
                                     ctypes.c_void_p(ext_out.data_ptr()) if ext else None, _stream_handle(stream)))


def propagate_noalloc(sys, psi, E, dt, nsteps, prec=FP64, obs=OBS_ALL, obs_out=None, dev_status=None,
                      stream=None):
    """tdsez_propagate_noalloc: the same propagation with no device
    allocation (working storage in the library's per-GPU scratch array);
    dev_status: device int32 tensor of 4 entries, or None."""
    import torch
    _check_dev(psi, torch.complex128)
    _check_dev(E, torch.float64)
    if obs:
        _check_dev(obs_out, torch.float64)
    if dev_status is not None:
        _check_dev(dev_status, torch.int32)
    _check(lib().tdsez_propagate_noalloc(sys.handle, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                         float(dt), int(nsteps), int(prec), int(obs),
                                         ctypes.c_void_p(obs_out.data_ptr()) if obs else None,
                                         None if dev_status is None else ctypes.c_void_p(dev_status.data_ptr()),
                                         _stream_handle(stream)))


def batch_status(batch, stream=None):
    s = ctypes.c_int()
    n = ctypes.c_int()
    _check(lib().tdsez_batch_status(batch.handle, _stream_handle(stream), ctypes.byref(s), ctypes.byref(n)))


def batch_profile(batch, stream=None):
    """Average cycles per step per phase, one row per system: (rhs, elim,
    fill, reduced, backsub, refine residual, refine reduced, refine backsub,
    partition count, largest relative refinement residual)."""
    out = np.zeros(PROFILE_COLUMNS * len(batch.systems))
    _check(lib().tdsez_batch_profile(batch.handle, _stream_handle(stream), _dptr(out)))
    return out.reshape(-1, PROFILE_COLUMNS)


def autotune(batch, prec=None, budget_ms=2000.0):
    """Choose every system's partition count by timing short propagations of
    the whole batch (tdsez_autotune); returns the chosen counts."""
    if prec is None:
        prec = FP32_REFINED
    _check(lib().tdsez_autotune(batch.handle, int(prec), float(budget_ms)))
    return batch_chunks(batch)


def batch_chunks(batch):
    """Partition count P of every system under the batch's current plan."""
    out = np.zeros(len(batch.systems), dtype=np.int32)
    _check(lib().tdsez_batch_chunks(batch.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return out


SPLIT_AUTO = -1


def batch_split(batch, nsteps, count):
    """Run the `count` systems with the largest N (p + 1) nsteps on two waves,
    or four with the batch key max_waves = 4 (nsteps may be None with
    count = 0; SPLIT_AUTO chooses the count from the device's SIMDs)."""
    if nsteps is None:
        _check(lib().tdsez_batch_split(batch.handle, None, int(count)))
        return
    ns = np.ascontiguousarray(nsteps, dtype=np.int32)
    if ns.shape != (len(batch.systems),):
        raise ValueError("nsteps must hold one count per system")
    _check(lib().tdsez_batch_split(batch.handle, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(count)))


def batch_two_wave(batch):
    """1 for every system running on more than one wave under the current plan."""
    out = np.zeros(len(batch.systems), dtype=np.int32)
    _check(lib().tdsez_batch_two_wave(batch.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return out


def batch_waves(batch):
    """Waves (1, 2 or 4) of every system under the current plan."""
    out = np.zeros(len(batch.systems), dtype=np.int32)
    _check(lib().tdsez_batch_waves(batch.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return out


def system_set(sys, key, value):
    """Partition settings of the single-system plan ("workgroups",
    "chunks_per_workgroup"; tdsez_system_set)."""
    _check(lib().tdsez_system_set(sys.handle, key.encode(), float(value)))


def system_workgroups(sys):
    """(workgroups, chunk count) of the single-system plan."""
    g, c = ctypes.c_int(), ctypes.c_int()
    _check(lib().tdsez_system_workgroups(sys.handle, ctypes.byref(g), ctypes.byref(c)))
    return g.value, c.value


def system_status(sys, stream=None):
    n = ctypes.c_int()
    _check(lib().tdsez_system_status(sys.handle, _stream_handle(stream), ctypes.byref(n)))


def pack_batch_inputs(systems_defs, psi0_list, device="cuda"):
    """Pack per-system initial states and pulse samples into the flat device
    buffers of propagate_batched; returns (psi, psi_off, E, E_off, obs, obs_off)."""
    import torch
    psi_off = np.cumsum([0] + [len(p) for p in psi0_list[:-1]]).astype(np.int64)
    E_off = np.cumsum([0] + [s.nsteps + 1 for s in systems_defs[:-1]]).astype(np.int64)
    obs_off = 3 * E_off
    psi = torch.from_numpy(np.concatenate(psi0_list).astype(np.complex128)).to(device)
    E = torch.from_numpy(np.concatenate([s.E[: s.nsteps + 1] for s in systems_defs]).astype(np.float64)).to(device)
    obs = torch.zeros(3 * int(E.numel()), dtype=torch.float64, device=device)
    return psi, psi_off, E, E_off, obs, obs_off


# --------------------------------------------------------------------- 2D
class System2D:
    """An assembled 2D tensor-product problem (owns its device data)."""

    def __init__(self, handle):
        self.handle = handle
        nx, ny, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().tdsez_system2d_size(handle, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(p)))
        self.Nx, self.Ny, self.p = nx.value, ny.value, p.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tdsez_system2d_destroy(self.handle)
            self.handle = None


def assemble_2d(breaks_x, breaks_y, order, nq, V_q, dVx_q=None):
    bx, by = _f64(breaks_x), _f64(breaks_y)
    vq = _f64(V_q)
    gq = None if dVx_q is None else _f64(dVx_q)
    h = ctypes.c_void_p()
    _check(lib().tdsez_assemble_2d(_dptr(bx), len(bx), _dptr(by), len(by), order, nq, _dptr(vq),
                                   _dptr(gq) if gq is not None else None, ctypes.byref(h)))
    return System2D(h)


def assemble_workload_2d(sysdef, with_force=True):
    """Assemble a workloads.System2D: sample V (and dV/dx, when the
    definition has it and with_force) on the tensor grid of the library's
    own per-axis quadrature points."""
    xq = quad_points(sysdef.breaks_x, sysdef.nq)
    yq = quad_points(sysdef.breaks_y, sysdef.nq)
    X, Y = np.meshgrid(xq, yq)
    g = sysdef.dVx(X, Y) if (with_force and sysdef.dVx is not None) else None
    return assemble_2d(sysdef.breaks_x, sysdef.breaks_y, sysdef.order, sysdef.nq, sysdef.V(X, Y), g)


def get_v2(sys2d):
    w = 2 * sys2d.p + 1
    out = np.zeros(sys2d.Nx * sys2d.Ny * w * w)
    _check(lib().tdsez_get_v2(sys2d.handle, _dptr(out)))
    return out.reshape(sys2d.Nx * sys2d.Ny, w, w)


def propagate_2d(sys2d, psi, E, dt, nsteps, prec=FP64, obs=OBS_NORM | OBS_DIPOLE, obs_out=None, tol=1e-12,
                 maxit=200, stream=None):
    """psi: device complex128 (Ny*Nx, in/out); E: device float64; obs_out:
    device float64 [(nsteps+1)*3] or None."""
    import torch
    _check_dev(psi, torch.complex128)
    _check_dev(E, torch.float64)
    if obs:
        _check_dev(obs_out, torch.float64)
    _check(lib().tdsez_propagate_2d(sys2d.handle, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                    float(dt), int(nsteps), int(prec), int(obs),
                                    ctypes.c_void_p(obs_out.data_ptr()) if obs else None, float(tol), int(maxit),
                                    _stream_handle(stream)))


def system2d_stats(sys2d):
    """(steps, Krylov iterations, largest iteration count of one step,
    refinement sweeps) since the last call."""
    a, b, c, d = ctypes.c_long(), ctypes.c_long(), ctypes.c_int(), ctypes.c_long()
    _check(lib().tdsez_system2d_stats(sys2d.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                      ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


# --------------------------------------------------------------------- 3D
class System3D:
    """An assembled 3D tensor-product problem (owns its device data)."""

    def __init__(self, handle):
        self.handle = handle
        nx, ny, nz, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().tdsez_system3d_size(handle, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(nz),
                                         ctypes.byref(p)))
        self.Nx, self.Ny, self.Nz, self.p = nx.value, ny.value, nz.value, p.value

    @property
    def N(self):
        return self.Nx * self.Ny * self.Nz

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tdsez_system3d_destroy(self.handle)
            self.handle = None


def assemble_3d(breaks_x, breaks_y, breaks_z, order, nq, V_q):
    """V_q: host samples at the tensor grid of the per-axis quadrature
    points, indexed [qz][qy][qx]."""
    bx, by, bz = _f64(breaks_x), _f64(breaks_y), _f64(breaks_z)
    vq = _f64(V_q)
    h = ctypes.c_void_p()
    _check(lib().tdsez_assemble_3d(_dptr(bx), len(bx), _dptr(by), len(by), _dptr(bz), len(bz), order, nq,
                                   _dptr(vq), ctypes.byref(h)))
    return System3D(h)


def sample_3d(V, xq, yq, zq):
    """V(x, y, z) on the tensor grid, [qz][qy][qx], one z plane at a time."""
    out = np.empty((len(zq), len(yq), len(xq)))
    Y, X = np.meshgrid(yq, xq, indexing="ij")
    for k, z in enumerate(zq):
        out[k] = V(X, Y, np.full_like(X, z))
    return out


def assemble_workload_3d(sysdef):
    """Assemble a workloads.System3D on the library's own per-axis
    quadrature points."""
    xq = quad_points(sysdef.breaks_x, sysdef.nq)
    yq = quad_points(sysdef.breaks_y, sysdef.nq)
    zq = quad_points(sysdef.breaks_z, sysdef.nq)
    return assemble_3d(sysdef.breaks_x, sysdef.breaks_y, sysdef.breaks_z, sysdef.order, sysdef.nq,
                       sample_3d(sysdef.V, xq, yq, zq))


def get_v3_rows(sys3d, rows):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    w = 2 * sys3d.p + 1
    out = np.zeros(len(rows) * w ** 3)
    _check(lib().tdsez_get_v3_rows(sys3d.handle, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(rows),
                                   _dptr(out)))
    return out.reshape(len(rows), w, w, w)


def apply_3d(sys3d, c, out, a, b, Ebar=0.0, stream=None):
    """out = a S3 c + b (T3 + V3 + Ebar D3) c (device complex128 vectors)."""
    import torch
    _check_dev(c, torch.complex128)
    _check_dev(out, torch.complex128)
    a, b = complex(a), complex(b)
    _check(lib().tdsez_apply_3d(sys3d.handle, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                a.real, a.imag, b.real, b.imag, float(Ebar), _stream_handle(stream)))


def propagate_3d(sys3d, psi, E, dt, nsteps, prec=FP64, obs=OBS_NORM | OBS_DIPOLE, obs_out=None, tol=1e-12,
                 maxit=200, stream=None):
    """psi: device complex128 (Nz*Ny*Nx, in/out); E: device float64; obs_out:
    device float64 [(nsteps+1)*3] or None."""
    import torch
    _check_dev(psi, torch.complex128)
    _check_dev(E, torch.float64)
    if obs:
        _check_dev(obs_out, torch.float64)
    _check(lib().tdsez_propagate_3d(sys3d.handle, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                    float(dt), int(nsteps), int(prec), int(obs),
                                    ctypes.c_void_p(obs_out.data_ptr()) if obs else None, float(tol), int(maxit),
                                    _stream_handle(stream)))


def system3d_stats(sys3d):
    """(steps, Krylov iterations, largest iteration count of one step,
    refinement sweeps) since the last call."""
    a, b, c, d = ctypes.c_long(), ctypes.c_long(), ctypes.c_int(), ctypes.c_long()
    _check(lib().tdsez_system3d_stats(sys3d.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                      ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def time_apply(sys_nd, prec=FP64, reps=20, stream=None):
    """Average ms per launch of the 2D or 3D operator kernel (HIP events)."""
    ms = ctypes.c_double()
    f = lib().tdsez_time_apply_3d if isinstance(sys_nd, System3D) else lib().tdsez_time_apply_2d
    _check(f(sys_nd.handle, int(prec), int(reps), _stream_handle(stream), ctypes.byref(ms)))
    return ms.value


def ground_state_3d(sys3d, sigma, tol=1e-12, maxit=60):
    """(energy, device complex128 eigenvector) of the lowest 3D level by
    shifted inverse iteration (sigma below that level)."""
    import torch
    psi = torch.zeros(sys3d.N, dtype=torch.complex128, device="cuda")
    e = ctypes.c_double()
    _check(lib().tdsez_ground_state_3d(sys3d.handle, float(sigma), float(tol), int(maxit),
                                       ctypes.c_void_p(psi.data_ptr()), ctypes.byref(e)))
    return e.value, psi
