"""Two-wave systems (tdsez_batch_split) on the GPU.

Marking a system for two waves changes its partition (up to 128 chunks)
and solves the separator system from both ends; the propagation must still
meet the oracle bars: FP64 1e-10 relative L2 on the state and every
observable series, FP32-refined 1e-5 on the series.  The two-wave launch
runs on the caller's stream beside a one-wave launch on an internal side
stream, so a graph captured from the call must replay to the eager result
bit for bit, and mixed batches must keep the per-system bookkeeping
(profile rows, chunk counts) in system order.  The adjoint runs the
two-wave systems on two waves and returns the one-wave batch's gradient to
rounding.
"""
import gc
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


def _mixed_batch(ns, seed=5):
    """Three of the largest and three of the smallest systems of a seeded
    uneven batch (N in 500..4000, orders 6..8), field on from step 0."""
    defs = W.config3(nsys=24, seed=seed)
    defs = sorted(defs, key=lambda s: -s.ndof)[:3] + sorted(defs, key=lambda s: s.ndof)[:3]
    for s in defs:
        s.nsteps = ns
        s.E = s.meta["E0"] * np.sin(s.meta["omega"] * s.dt * np.arange(ns + 1) + 0.4)
    return defs


def _check(defs, refs, psi, po, obs, eo, ns, tol_state, tol_obs):
    o = obs.cpu().numpy()
    c = psi.cpu().numpy()
    for i, (r, cr) in enumerate(refs):
        gi = o[3 * eo[i]: 3 * eo[i] + 3 * (ns + 1)].reshape(-1, 3)
        if tol_state is not None:
            assert rel(c[po[i]: po[i] + len(cr)], cr) < tol_state, i
        errs = [rel(gi[:, k], r[:, k]) for k in range(3)]
        say("system", i, "N", defs[i].ndof, "errors", errs)
        for k in range(3):
            assert errs[k] < tol_obs, (i, k, errs[k])


@pytest.mark.parametrize("prec", [T.FP64, T.FP32_REFINED])
def test_two_wave_systems_match_oracle(prec):
    ns = 60
    defs = _mixed_batch(ns)
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    one = T.batch_chunks(b).copy()
    T.batch_split(b, [ns] * len(defs), 3)
    flags = T.batch_two_wave(b)
    chunks = T.batch_chunks(b)
    say("one-wave chunks", one.tolist(), "two-wave flags", flags.tolist(), "chunks", chunks.tolist())
    # the three largest systems (N > 3000) get more than 64 chunks
    assert flags.tolist() == [1, 1, 1, 0, 0, 0]
    assert np.all(chunks[:3] > 64) and np.all(chunks[:3] <= 128)
    assert np.array_equal(chunks[3:], one[3:])
    refs, psi0s = [], []
    for s in defs:
        m, p0 = _oracle(s)
        psi0s.append(p0)
        refs.append(O.propagate(m, p0, s.E, s.dt, ns))
    T.batch_set(b, "profile", 1)
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, psi0s)
    T.propagate_batched(b, psi, po, E, eo, [s.dt for s in defs], [ns] * len(defs), prec, T.OBS_ALL, obs, oo)
    T.batch_status(b)
    prof = T.batch_profile(b)
    assert np.array_equal(prof[:, 8].astype(int), chunks)
    if prec == T.FP64:
        _check(defs, refs, psi, po, obs, eo, ns, 1e-10, 1e-10)
    else:
        _check(defs, refs, psi, po, obs, eo, ns, None, 1e-5)
    # count = 0 restores one wave per system
    T.batch_split(b, None, 0)
    assert T.batch_two_wave(b).tolist() == [0] * len(defs)
    assert np.array_equal(T.batch_chunks(b), one)


def test_two_wave_autotune_and_adjoint():
    ns = 40
    defs = _mixed_batch(ns, seed=6)
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    T.batch_split(b, [ns] * len(defs), 2)
    tuned = T.autotune(b, T.FP64, 1200.0)
    flags = T.batch_two_wave(b)
    say("tuned", tuned.tolist(), "flags", flags.tolist())
    assert np.all(tuned >= 1) and np.all(tuned <= 128)
    assert np.all((tuned > 64) == (flags == 1))
    assert flags.sum() <= 2
    refs, psi0s = [], []
    for s in defs:
        m, p0 = _oracle(s)
        psi0s.append(p0)
        refs.append(O.propagate(m, p0, s.E, s.dt, ns))
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, psi0s)
    dts = [s.dt for s in defs]
    T.propagate_batched(b, psi, po, E, eo, dts, [ns] * len(defs), T.FP64, T.OBS_ALL, obs, oo)
    T.batch_status(b)
    _check(defs, refs, psi, po, obs, eo, ns, 1e-10, 1e-10)
    if flags.sum() > 0:
        # the adjoint runs the two-wave systems on two waves: the gradient
        # equals the one-wave batch's to rounding
        psi_in, _, _, _, _, _ = T.pack_batch_inputs(defs, psi0s)
        dJ = torch.from_numpy(np.random.default_rng(9).normal(size=obs.numel())).cuda()
        dE2 = torch.zeros_like(E)
        T.adjoint_batched(b, psi_in, po, E, eo, dts, [ns] * len(defs), T.OBS_ALL, dJ, oo, dE2)
        T.batch_status(b)
        b1 = T.batch_create([T.assemble_workload(s) for s in defs])
        dE1 = torch.zeros_like(E)
        T.adjoint_batched(b1, psi_in, po, E, eo, dts, [ns] * len(defs), T.OBS_ALL, dJ, oo, dE1)
        T.batch_status(b1)
        g1, g2 = dE1.cpu().numpy(), dE2.cpu().numpy()
        for i in range(len(defs)):
            sl_ = slice(eo[i], eo[i] + ns + 1)
            say("adjoint system", i, "two-wave" if flags[i] else "one-wave", rel(g2[sl_], g1[sl_]))
            assert rel(g2[sl_], g1[sl_]) < 1e-9, i
    with pytest.raises(T.TdsezError) as e:
        T.batch_split(b, [ns] * len(defs), len(defs) + 1)
    assert e.value.status == 1


@pytest.mark.parametrize("prec", [T.FP64, T.FP32_REFINED])
def test_two_wave_graph_replays_match_eager(prec):
    ns = 50
    defs = _mixed_batch(ns, seed=7)
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    T.batch_split(b, [ns] * len(defs), 3)
    assert T.batch_two_wave(b).sum() >= 1
    psi0, po, E, eo, obs, oo = T.pack_batch_inputs(defs, [np.zeros(s.ndof) for s in defs])
    T.ground_state_batched(b, psi0, po)
    dts = [s.dt for s in defs]
    nss = [ns] * len(defs)
    psi_ref = psi0.clone()
    obs_ref = torch.zeros_like(obs)
    T.propagate_batched(b, psi_ref, po, E, eo, dts, nss, prec, T.OBS_ALL, obs_ref, oo)
    T.batch_status(b)
    torch.cuda.synchronize()
    psi = psi0.clone()
    ob = torch.zeros_like(obs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        T.propagate_batched(b, psi, po, E, eo, dts, nss, prec, T.OBS_ALL, ob, oo, side)  # warm-up
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    psi.copy_(psi0)
    torch.cuda.synchronize()
    # handles of earlier tests must not be destroyed (device frees) while
    # the capture runs: collect them now and keep the collector off
    gc.collect()
    gc.disable()
    try:
        with torch.cuda.graph(graph):
            T.propagate_batched(b, psi, po, E, eo, dts, nss, prec, T.OBS_ALL, ob, oo, torch.cuda.current_stream())
    finally:
        gc.enable()
    for rep in range(3):
        psi.copy_(psi0)
        ob.zero_()
        scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        scratch.mul_(2.0).sum().item()
        graph.replay()
        torch.cuda.synchronize()
        T.batch_status(b)
        dpsi = float((psi - psi_ref).abs().max())
        dobs = float((ob - obs_ref).abs().max())
        say("replay", rep, dpsi, dobs)
        assert dpsi == 0.0 and dobs == 0.0


def test_all_two_wave_batch_odd_chunks_and_zero_steps():
    """Every system on two waves (the one-wave launch is empty), an odd
    chunk count (the backward half of the separator chain holds one block
    more than the forward half) and per-system step counts 0, 25 and 40;
    FP64 against the oracle."""
    V, dV = W.soft_coulomb(2.0)
    defs = []
    for n_el, order, ns in ((1270, 7, 25), (1600, 8, 0), (2300, 6, 40)):
        E = 0.06 * np.sin(0.05 * 0.05 * np.arange(ns + 1) + 0.4)
        defs.append(W.System("two-%d" % n_el, W.breaks_uniform(200.0, n_el - order + 3), order,
                             lambda x: np.ones_like(x), V, dV, 10, E, 0.05, ns, True))
    b = T.batch_create([T.assemble_workload(s) for s in defs])
    nss = [s.nsteps for s in defs]
    T.batch_split(b, nss, len(defs))
    chunks = T.batch_chunks(b)
    say("N", [s.ndof for s in defs], "chunks", chunks.tolist())
    assert T.batch_two_wave(b).tolist() == [1, 1, 1]
    assert chunks[0] % 2 == 1
    refs, psi0s = [], []
    for s in defs:
        m, p0 = _oracle(s)
        psi0s.append(p0)
        refs.append(O.propagate(m, p0, s.E, s.dt, s.nsteps))
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, psi0s)
    T.propagate_batched(b, psi, po, E, eo, [s.dt for s in defs], nss, T.FP64, T.OBS_ALL, obs, oo)
    T.batch_status(b)
    o = obs.cpu().numpy()
    c = psi.cpu().numpy()
    for i, (r, cr) in enumerate(refs):
        ns = defs[i].nsteps
        gi = o[3 * eo[i]: 3 * eo[i] + 3 * (ns + 1)].reshape(-1, 3)
        assert rel(c[po[i]: po[i] + len(cr)], cr) < 1e-10, i
        say("system", i, "steps", ns, "max |obs - oracle|", np.abs(gi - r).max(0).tolist())
        if ns == 0:
            # only the initial state's observables: its dipole and acceleration
            # vanish up to rounding (symmetric potential and knots), so they are
            # compared in absolute terms
            assert np.abs(gi - r).max() < 1e-12, i
            continue
        for k in range(3):
            assert rel(gi[:, k], r[:, k]) < 1e-10, (i, k)


@pytest.mark.parametrize("P", [66, 67, 70, 71])
def test_forced_two_wave_chunk_counts(P):
    """Forced two-wave chunk counts whose halves (P/2 forward, the rest
    backward) leave every remainder of the separator chain's four-block
    prefetch groups (two in FP64); both precisions against the oracle."""
    ns = 40
    V, dV = W.soft_coulomb(2.0)
    E = 0.06 * np.sin(0.05 * 0.05 * np.arange(ns + 1) + 0.4)
    sd = W.System("two-forced", W.breaks_uniform(300.0, 3000 - 8 + 3), 8, lambda x: np.ones_like(x), V, dV, 10,
                  E, 0.05, ns, True)
    b = T.batch_create([T.assemble_workload(sd)])
    T.batch_split(b, [ns], 1)
    T.batch_set(b, "chunks", P)
    assert T.batch_two_wave(b).tolist() == [1]
    assert T.batch_chunks(b).tolist() == [P]
    m, p0 = _oracle(sd)
    r, cr = O.propagate(m, p0, sd.E, sd.dt, ns)
    for prec in (T.FP64, T.FP32_REFINED):
        psi, po, Eb, eo, obs, oo = T.pack_batch_inputs([sd], [p0])
        T.propagate_batched(b, psi, po, Eb, eo, [sd.dt], [ns], prec, T.OBS_ALL, obs, oo)
        T.batch_status(b)
        got = obs.cpu().numpy().reshape(-1, 3)
        errs = [rel(got[:, k], r[:, k]) for k in range(3)]
        es = rel(psi.cpu().numpy(), cr)
        say("P", P, "prec", prec, "state", es, "series", errs)
        if prec == T.FP64:
            assert es < 1e-10 and max(errs) < 1e-10
        else:
            assert max(errs) < 1e-5


def test_automatic_split_count_fills_the_simds():
    """SPLIT_AUTO marks clamp(floor(1.16 S) - nsys, 0, nsys) systems, S = 4 x
    the device's compute units; every marked system of N = 1600 (73 chunks
    on two waves) runs on two waves, the costliest first."""
    S = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    V, dV = W.soft_coulomb(2.0)
    for nsys in (int(1.16 * S) - 150, 3):
        defs = []
        for i in range(nsys):
            ns = 10 + (i % 7)
            E = np.zeros(ns + 1)
            defs.append(W.System("auto-%d" % i, W.breaks_uniform(200.0, 1600 - 8 + 3), 8, lambda x: np.ones_like(x),
                                 V, dV, 10, E, 0.05, ns, True))
        b = T.batch_create([T.assemble_workload(d) for d in defs])
        T.batch_split(b, [d.nsteps for d in defs], T.SPLIT_AUTO)
        flags = T.batch_two_wave(b)
        want = max(0, min(nsys, int(1.16 * S) - nsys))
        say("nsys", nsys, "S", S, "two-wave", int(flags.sum()), "expected", want)
        assert int(flags.sum()) == want
        if 0 < want < nsys:
            # the marked systems are those with the most steps (same N and p)
            ns = np.array([d.nsteps for d in defs])
            assert ns[flags == 1].min() >= ns[flags == 0].max()


def test_marked_small_system_keeps_its_one_wave_plan():
    """A system marked for two waves whose two-wave plan has at most 64
    chunks (N = 1004: 58) keeps the one-wave plan (41 chunks)."""
    sd = W.config1(nsteps=4)
    b = T.batch_create([T.assemble_workload(sd)])
    one = T.batch_chunks(b).copy()
    T.batch_split(b, [4], 1)
    assert T.batch_two_wave(b).tolist() == [0]
    assert np.array_equal(T.batch_chunks(b), one)


def test_single_system_runs_on_two_waves():
    """tdsez_propagate on a system above the two-wave threshold (N = 2000):
    FP64 and FP32-refined against the oracle over 200 steps."""
    V, dV = W.soft_coulomb(2.0)
    ns = 200
    E = 0.06 * np.sin(0.05 * 0.05 * np.arange(ns + 1) + 0.4)
    sd = W.System("lone", W.breaks_uniform(200.0, 2000 - 8 + 3), 8, lambda x: np.ones_like(x), V, dV, 10, E,
                  0.05, ns, True)
    g = T.assemble_workload(sd)
    m, p0 = _oracle(sd)
    ref, cref = O.propagate(m, p0, sd.E, sd.dt, ns)
    for prec, tol in ((T.FP64, 1e-10), (T.FP32_REFINED, 1e-5)):
        psi = torch.from_numpy(p0.copy()).cuda()
        Et = torch.from_numpy(E.copy()).cuda()
        o = torch.zeros(3 * (ns + 1), dtype=torch.float64, device="cuda")
        T.propagate(g, psi, Et, sd.dt, ns, prec, T.OBS_ALL, o)
        T.system_status(g)
        got = o.cpu().numpy().reshape(-1, 3)
        errs = [rel(got[:, k], ref[:, k]) for k in range(3)]
        say("lone system", sd.ndof, prec, errs)
        assert max(errs) < tol
        if prec == T.FP64:
            assert rel(psi.cpu().numpy(), cref) < 1e-10
