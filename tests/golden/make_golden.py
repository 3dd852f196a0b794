"""Writes the oracle's stored series used by the full-scale GPU parity tests.

Every value written here comes from oracle/ (the serial FP64 C oracle and
its NumPy 2D front-end) fed by paper_2608_18472_amd.workloads; nothing is
taken from the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py batch32      # ~1 min on 8 cores
    python tests/golden/make_golden.py config4_128  # whole 128 x 128 pulse, ~20 min
    python tests/golden/make_golden.py config4_512  # 200 steps of 512 x 512, ~10 min
    python tests/golden/make_golden.py config5      # full-size adjoint + FD, ~5 min

Outputs (next to this script):
  batch32_fullpulse.npz   the 32-system subset of the 1024-system batch
                          (indices, ground-state energies, whole-pulse dipole)
  config4_128_fullpulse.npz  nu and x-dipole over all 8819 steps, 128 x 128
  config4_512_segment.npz    nu and x-dipole over steps 2000..2200 of the pulse
                             (field on) from the product ground state, 512 x 512
  config5_adjoint.json    dJ/dtheta of the Fourier-pulse harmonic yield for 4
                          full config-5 systems (oracle adjoint) and central
                          differences of J on 2 systems x 4 amplitudes
"""
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2608_18472_amd import workloads as W  # noqa: E402


def shift_of(sd):
    xq, _ = O.quad_points(sd.breaks, sd.nq)
    vmin = float(np.min(sd.V(xq)))
    return vmin - 1e-3 * (abs(vmin) + 1.0)


def batch32_pick():
    """The seeded 32-system subset: smallest and largest N, the first system
    of every order, the rest drawn from default_rng(5)."""
    defs_all = W.config3(nsys=1024, seed=0)
    order = np.argsort([s.ndof for s in defs_all])
    rng = np.random.default_rng(5)
    pick = {int(order[0]), int(order[-1])}
    for k in (6, 7, 8):
        pick.add(int(next(i for i in order if defs_all[i].order == k)))
    while len(pick) < 32:
        pick.add(int(rng.integers(0, 1024)))
    return sorted(pick)


def _batch_one(idx):
    sd = W.config3(nsys=1024, seed=0)[idx]
    m = O.assemble(sd.breaks, sd.order, sd.nq, None, sd.V, sd.dV)
    ev, vec = O.eig_banded(m["H0"], m["S"], 1, shift_of(sd))
    ref, _ = O.propagate(m, vec[0].astype(np.complex128), sd.E, sd.dt, sd.nsteps)
    return idx, float(ev[0]), ref


def make_batch32():
    pick = batch32_pick()
    t0 = time.time()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(_batch_one, pick)
    res.sort()
    lens = [r[2].shape[0] for r in res]
    dipole = np.concatenate([r[2][:, 1] for r in res])
    np.savez_compressed(os.path.join(HERE, "batch32_fullpulse.npz"), pick=np.array(pick),
                        eps0=np.array([r[1] for r in res]), lens=np.array(lens), dipole=dipole,
                        command="python tests/golden/make_golden.py batch32")
    print("batch32 done in %.1f s" % (time.time() - t0))


def product_ground_state(sd):
    vecs = []
    for br in (sd.breaks_x, sd.breaks_y):
        m = O.assemble(br, sd.order, sd.nq, V=lambda x: -1.0 / np.sqrt(x * x + 1.0))
        ev, vec = O.eig_banded(m["H0"], m["S"], 1, -1.5)
        vecs.append(vec[0])
    return np.outer(vecs[1], vecs[0]).astype(np.complex128)


def make_config4(n, n0, nsteps, name):
    sd = W.config4(n=n)
    m2 = O.assemble_2d(sd.breaks_x, sd.breaks_y, sd.order, sd.nq, sd.V)
    psi0 = product_ground_state(sd)
    E = np.ascontiguousarray(sd.E[n0: n0 + nsteps + 1])
    t0 = time.time()
    obs, _ = O.propagate_2d(m2, psi0, E, sd.dt, nsteps, tol=1e-14)
    np.savez_compressed(os.path.join(HERE, name), n=n, n0=n0, nsteps=nsteps, obs=obs, tol=1e-14,
                        command="python tests/golden/make_golden.py %s" % sys.argv[1])
    print("%s done in %.1f s" % (name, time.time() - t0))


C5_SYSTEMS = (0, 21, 42, 63)
C5_FD = ((0, 15), (0, 3), (21, 40), (21, 7))


def _c5_setup():
    defs, thetas, basis = W.config5()
    m = O.assemble(defs[0].breaks, defs[0].order, defs[0].nq, defs[0].minv, defs[0].V, defs[0].dV)
    ev, vec = O.eig_banded(m["H0"], m["S"], 2, shift_of(defs[0]))
    return defs, thetas, basis, m, vec[0].astype(np.complex128)


def _c5_J(args):
    """J(theta) of one system from the oracle's forward dipole series."""
    import torch
    s, theta = args
    defs, thetas, basis, m, psi0 = _c5_setup()
    sd = defs[s]
    ser, _ = O.propagate(m, psi0, basis @ theta, sd.dt, sd.nsteps, with_accel=False)
    return float(W.harmonic_yield(torch.from_numpy(ser[:, 1].copy()), sd.dt, sd.meta["omega"]))


def _c5_grad(s):
    import torch
    defs, thetas, basis, m, psi0 = _c5_setup()
    sd = defs[s]
    E = basis @ thetas[s]
    ser, _ = O.propagate(m, psi0, E, sd.dt, sd.nsteps, with_accel=False)
    d = torch.from_numpy(ser[:, 1].copy()).requires_grad_(True)
    J = W.harmonic_yield(d, sd.dt, sd.meta["omega"])
    J.backward()
    dJ = np.zeros((sd.nsteps + 1, 3))
    dJ[:, 1] = d.grad.numpy()
    gE, _ = O.adjoint(m, psi0, E, sd.dt, sd.nsteps, dJ, with_accel=False)
    return s, float(J.detach()), (basis.T @ gE).tolist()


def make_config5():
    t0 = time.time()
    defs, thetas, basis, m, psi0 = _c5_setup()
    h = 1e-4 * float(np.abs(thetas).max())
    jobs = []
    for s, j in C5_FD:
        for sg in (1.0, -1.0):
            th = thetas[s].copy()
            th[j] += sg * h
            jobs.append((s, th))
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        grads = pool.map(_c5_grad, C5_SYSTEMS)
        Js = pool.map(_c5_J, jobs)
    fd = []
    for k, (s, j) in enumerate(C5_FD):
        fd.append({"system": s, "theta": j, "dJ": (Js[2 * k] - Js[2 * k + 1]) / (2 * h)})
    out = {"command": "python tests/golden/make_golden.py config5",
           "workload": "config5(): 64 double-quantum-well systems, N 1500, 20000 steps, 64 Fourier amplitudes; "
                       "initial state = oracle ground state (nev 2), objective W.harmonic_yield of the dipole",
           "fd_step": h,
           "systems": [{"index": s, "J": J, "dJdtheta": g} for s, J, g in grads],
           "finite_differences": fd}
    with open(os.path.join(HERE, "config5_adjoint.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("config5 done in %.1f s" % (time.time() - t0))


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "batch32":
        make_batch32()
    elif what == "config4_128":
        make_config4(128, 0, W.config4(n=128).nsteps, "config4_128_fullpulse.npz")
    elif what == "config4_512":
        make_config4(512, 2000, 200, "config4_512_segment.npz")
    elif what == "config5":
        make_config5()
    else:
        raise SystemExit("unknown target " + what)
