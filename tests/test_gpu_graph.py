"""The batched propagation captured into a HIP graph (torch.cuda.CUDAGraph)
and replayed: every replay, with eager work on the same stream in between,
must reproduce the eager result bit for bit (same kernels, fixed summation
order).  A warm-up call with the same arguments precedes the capture, so the
captured call enqueues kernels only."""
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


@pytest.mark.parametrize("prec", [T.FP64, T.FP32_REFINED])
def test_graph_replays_match_eager(prec):
    defs = W.config3(nsys=6, seed=4)
    ns = 80
    for s in defs:
        s.nsteps = ns
        s.E = s.meta["E0"] * np.sin(s.meta["omega"] * s.dt * np.arange(ns + 1))
    gs = [T.assemble_workload(s) for s in defs]
    b = T.batch_create(gs)
    psi0, po, E, eo, obs, oo = T.pack_batch_inputs(defs, [np.zeros(s.ndof) for s in defs])
    T.ground_state_batched(b, psi0, po)
    dts = [s.dt for s in defs]
    nss = [ns] * len(defs)
    # eager reference
    psi_ref = psi0.clone()
    obs_ref = torch.zeros_like(obs)
    T.propagate_batched(b, psi_ref, po, E, eo, dts, nss, prec, T.OBS_ALL, obs_ref, oo)
    T.batch_status(b)
    torch.cuda.synchronize()
    # buffers owned by the graph
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
        # unrelated eager work on the stream between replays
        scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        scratch.mul_(2.0).sum().item()
        graph.replay()
        torch.cuda.synchronize()
        T.batch_status(b)
        dpsi = float((psi - psi_ref).abs().max())
        dobs = float((ob - obs_ref).abs().max())
        say("replay", rep, dpsi, dobs)
        assert dpsi == 0.0 and dobs == 0.0
