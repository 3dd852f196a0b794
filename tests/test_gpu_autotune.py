"""Partition autotuner and longest-first dispatch on the GPU.

The tuned plan changes only how each system is partitioned, so propagation
with it must still match the FP64 oracle to the FP64 bar (1e-10 relative L2
on every observable series); the profile and chunk queries must report the
plan per system whatever order the workgroups run in.
"""
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


def _oracle(sd):
    m = O.assemble(sd.breaks, sd.order, sd.nq, None, sd.V, sd.dV)
    xq, _ = O.quad_points(sd.breaks, sd.nq)
    vmin = float(np.min(sd.V(xq)))
    ev, vec = O.eig_banded(m["H0"], m["S"], 1, vmin - 1e-3 * (abs(vmin) + 1.0))
    return m, vec[0].astype(np.complex128)


def test_autotune_plan_and_parity():
    defs = W.config3(nsys=16, seed=3)
    defs = sorted(defs, key=lambda s: s.ndof)[:4] + sorted(defs, key=lambda s: -s.ndof)[:4]
    ns = 60
    for s in defs:
        s.nsteps = ns
        s.E = s.meta["E0"] * np.sin(s.meta["omega"] * s.dt * np.arange(ns + 1))
    say("systems", [(s.ndof, s.order) for s in defs])
    gs = [T.assemble_workload(s) for s in defs]
    b = T.batch_create(gs)
    rule = T.batch_chunks(b).copy()
    tuned = T.autotune(b, T.FP64, 1500.0)
    say("rule", rule.tolist(), "tuned", tuned.tolist())
    assert tuned.shape == rule.shape
    assert np.all(tuned >= 1) and np.all(tuned <= 64)
    assert np.array_equal(tuned, T.batch_chunks(b))
    refs = []
    psi0s = []
    for s in defs:
        m, p0 = _oracle(s)
        psi0s.append(p0)
        refs.append(O.propagate(m, p0, s.E, s.dt, ns))
    T.batch_set(b, "profile", 1)
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, psi0s)
    T.propagate_batched(b, psi, po, E, eo, [s.dt for s in defs], [ns] * len(defs), T.FP64, T.OBS_ALL, obs, oo)
    T.batch_status(b)
    prof = T.batch_profile(b)
    # profile rows follow the system index, not the dispatch order
    assert np.array_equal(prof[:, 8].astype(int), tuned)
    o = obs.cpu().numpy()
    c = psi.cpu().numpy()
    for i, (r, cr) in enumerate(refs):
        gi = o[3 * eo[i]: 3 * eo[i] + 3 * (ns + 1)].reshape(-1, 3)
        assert rel(c[po[i]: po[i] + len(cr)], cr) < 1e-10, i
        for k in range(3):
            assert rel(gi[:, k], r[:, k]) < 1e-10, (i, k, rel(gi[:, k], r[:, k]))
    # the explicit knob overrides the tuned plan
    T.batch_set(b, "chunks", 3)
    assert np.all(T.batch_chunks(b) <= 3)


def test_autotune_rejects_bad_arguments():
    defs = W.config3(nsys=2, seed=0)
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    with pytest.raises(T.TdsezError):
        T.autotune(b, T.FP64, 0.0)
    with pytest.raises(T.TdsezError):
        T.autotune(b, 7, 100.0)
