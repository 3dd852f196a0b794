"""Full-scale parity: the GPU path against the oracle's stored series at the
workloads' real sizes, plus the plateau-band harmonic-spectrum error.

Stored series (tests/golden/, written by tests/golden/make_golden.py from
the oracle only):
  - 32 systems of the 1024-system batch over their whole pulses;
  - the 2D workload on its 128 x 128 reduced grid over the whole 8819-step
    pulse, and on the full 512 x 512 grid over 200 field-on steps;
  - the pulse-amplitude gradient of 4 full double-quantum-well systems
    (N 1500, 20 000 steps, 64 amplitudes) and central differences on 2 x 4
    amplitudes.
Bars: FP64 <= 1e-10 relative L2 (gradient: <= 1e-9, the adjoint of a
20 000-step recursion is compared through the FFT objective on two
devices), FP32-refined <= 1e-5; spectrum error <= 0.01 dex over the odd
harmonics 3 .. q_cut + 6 (Kaiser window, beta 8).
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_18472_amd import spectrum as SP
from paper_2608_18472_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_18472_amd import tdsez as T  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import make_golden as MG  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def q_cut(sd, eps0):
    return SP.cutoff_order(-eps0, sd.meta["E0"], sd.meta["omega"])


def test_batch_subset_whole_pulses_and_spectra():
    """32 systems of the uneven batch (smallest and largest N, every order)
    in one persistent launch over their whole pulses (6 284 .. 16 756
    steps): dipole series against the oracle, FP64 and FP32-refined, and the
    plateau-band spectrum error of both."""
    z = np.load(os.path.join(GOLDEN, "batch32_fullpulse.npz"))
    pick, eps0, lens = z["pick"], z["eps0"], z["lens"]
    ref_d = np.split(z["dipole"], np.cumsum(lens)[:-1])
    defs_all = W.config3(nsys=1024, seed=0)
    defs = [defs_all[i] for i in pick]
    assert [s.nsteps + 1 for s in defs] == list(lens)
    psi0s = []
    for s in defs:
        m = O.assemble(s.breaks, s.order, s.nq, None, s.V, s.dV)
        ev, vec = O.eig_banded(m["H0"], m["S"], 1, MG.shift_of(s))
        psi0s.append(vec[0].astype(np.complex128))
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    worst = {}
    for prec, tol in ((T.FP64, 1e-10), (T.FP32_REFINED, 1e-5)):
        psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, psi0s)
        T.propagate_batched(b, psi, po, E, eo, [s.dt for s in defs], [s.nsteps for s in defs], prec, T.OBS_ALL,
                            obs, oo)
        T.batch_status(b)
        o = obs.cpu().numpy()
        ed, es = 0.0, 0.0
        for j, s in enumerate(defs):
            d = o[3 * eo[j]: 3 * eo[j] + 3 * (s.nsteps + 1)].reshape(-1, 3)[:, 1]
            e = rel(d, ref_d[j])
            assert e < tol, (prec, int(pick[j]), e)
            sp = SP.plateau_error(d, ref_d[j], s.dt, s.meta["omega"], q_cut(s, eps0[j]))
            assert sp <= 0.01, (prec, int(pick[j]), sp)
            ed, es = max(ed, e), max(es, sp)
        worst[prec] = (ed, es)
    say("worst dipole error / spectrum error (dex):", worst)


def test_full_batch_fp32_refined_spectra_match_fp64():
    """All 1024 systems, whole pulses, GPU ground states: the FP32-refined
    dipole series and harmonic spectra against the FP64 GPU path."""
    defs = W.config3(nsys=1024, seed=0)
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, [np.zeros(s.ndof) for s in defs])
    eps = T.ground_state_batched(b, psi, po)
    psi0 = psi.clone()
    series = {}
    for prec in (T.FP64, T.FP32_REFINED):
        psi.copy_(psi0)
        T.propagate_batched(b, psi, po, E, eo, [s.dt for s in defs], [s.nsteps for s in defs], prec, T.OBS_ALL,
                            obs, oo)
        T.batch_status(b)
        series[prec] = obs.cpu().numpy()
    ed, es = 0.0, 0.0
    for j, s in enumerate(defs):
        sl = slice(3 * eo[j], 3 * eo[j] + 3 * (s.nsteps + 1))
        d64 = series[T.FP64][sl].reshape(-1, 3)[:, 1]
        d32 = series[T.FP32_REFINED][sl].reshape(-1, 3)[:, 1]
        ed = max(ed, rel(d32, d64))
        es = max(es, SP.plateau_error(d32, d64, s.dt, s.meta["omega"], q_cut(s, eps[j])))
    say("1024 systems: worst FP32-refined vs FP64 dipole error %.3g, spectrum error %.3g dex" % (ed, es))
    assert ed < 1e-5
    assert es <= 0.01


def _product_state(sd):
    return MG.product_ground_state(sd)


def _run_2d(sd, psi0, E, nsteps, prec):
    g = T.assemble_workload_2d(sd)
    psi = torch.from_numpy(psi0.reshape(-1).copy()).cuda()
    Et = torch.from_numpy(np.ascontiguousarray(E[: nsteps + 1])).cuda()
    o = torch.zeros(3 * (nsteps + 1), dtype=torch.float64, device="cuda")
    T.propagate_2d(g, psi, Et, sd.dt, nsteps, prec, T.OBS_NORM | T.OBS_DIPOLE, o, tol=1e-13, maxit=300)
    return o.cpu().numpy().reshape(-1, 3)


@pytest.mark.parametrize("prec,tol", [(T.FP64, 1e-10), (T.FP32_REFINED, 1e-5)])
def test_2d_reduced_grid_whole_pulse(prec, tol):
    """128 x 128 reduced grid of the 2D workload over all 8819 steps of its
    pulse (norm and x dipole)."""
    z = np.load(os.path.join(GOLDEN, "config4_128_fullpulse.npz"))
    sd = W.config4(n=int(z["n"]))
    ns = int(z["nsteps"])
    assert ns == sd.nsteps
    got = _run_2d(sd, _product_state(sd), sd.E, ns, prec)
    ref = z["obs"]
    e = [rel(got[:, k], ref[:, k]) for k in (0, 1)]
    say("2D 128^2 whole pulse", prec, e)
    assert e[0] < tol and e[1] < tol


@pytest.mark.parametrize("prec,tol", [(T.FP64, 1e-10), (T.FP32_REFINED, 1e-5)])
def test_2d_full_grid_200_steps(prec, tol):
    """The full 512 x 512 grid over steps 2000..2200 of the pulse (field on)
    from the product ground state."""
    z = np.load(os.path.join(GOLDEN, "config4_512_segment.npz"))
    sd = W.config4(n=int(z["n"]))
    n0, ns = int(z["n0"]), int(z["nsteps"])
    got = _run_2d(sd, _product_state(sd), sd.E[n0:], ns, prec)
    ref = z["obs"]
    e = [rel(got[:, k], ref[:, k]) for k in (0, 1)]
    say("2D 512^2 segment", prec, e)
    assert e[0] < tol and e[1] < tol


def test_config5_full_size_gradient():
    """The pulse-gradient workload at full size: 64 double-quantum-well
    systems, N 1500, 20 000 steps, 64 Fourier amplitudes each, in one
    batch; dJ/dtheta through the differentiable series (GPU adjoint with
    sqrt(Nt) checkpoints) against the oracle's adjoint on 4 systems and
    central differences of the oracle's J on 2 x 4 amplitudes."""
    with open(os.path.join(GOLDEN, "config5_adjoint.json")) as f:
        gold = json.load(f)
    defs, thetas, basis = W.config5()
    m = O.assemble(defs[0].breaks, defs[0].order, defs[0].nq, defs[0].minv, defs[0].V, defs[0].dV)
    ev, vec = O.eig_banded(m["H0"], m["S"], 2, MG.shift_of(defs[0]))
    psi0 = vec[0].astype(np.complex128)
    omega = defs[0].meta["omega"]
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, [psi0] * len(defs))
    Bt = torch.from_numpy(basis).cuda()
    dt = [s.dt for s in defs]
    ns = [s.nsteps for s in defs]
    th = torch.from_numpy(thetas.copy()).cuda().requires_grad_(True)
    Ep = torch.cat([Bt @ th[i] for i in range(len(defs))])
    ser = T.observable_series(Ep, b, psi, po, eo, dt, ns, oo, T.OBS_NORM | T.OBS_DIPOLE)
    J = 0.0
    Js = []
    for i in range(len(defs)):
        d = ser[oo[i]: oo[i] + 3 * (ns[i] + 1)].reshape(-1, 3)[:, 1]
        Ji = W.harmonic_yield(d, dt[i], omega)
        Js.append(float(Ji.detach()))
        J = J + Ji
    J.backward()
    g = th.grad.cpu().numpy()
    gmax = max(np.abs(np.array(s["dJdtheta"])).max() for s in gold["systems"])
    for s in gold["systems"]:
        i = s["index"]
        e = rel(g[i], np.array(s["dJdtheta"]))
        ej = abs(Js[i] - s["J"]) / abs(s["J"])
        say("system", i, "gradient rel error", e, "J rel error", ej)
        assert ej < 1e-10
        assert e < 1e-9
    for f in gold["finite_differences"]:
        diff = abs(f["dJ"] - g[f["system"], f["theta"]])
        say("fd", f["system"], f["theta"], f["dJ"], g[f["system"], f["theta"]], diff / gmax)
        assert diff <= 1e-6 * gmax
