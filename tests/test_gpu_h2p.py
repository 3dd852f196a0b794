"""The 1D H2+ workload (30 007 degree-7 splines, one long chain) on the GPU.

A single system of this size runs on two waves with the 128-chunk cap
(235-row chunks).  Bars: eigenvalues 1e-12 relative against the oracle;
propagation over a flat-top segment of the trapezoidal pulse, FP64 1e-10 and
FP32-refined 1e-5 relative L2 on the norm and dipole series, FP64 1e-10 on
the final state.
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


def test_h2p_long_chain_matches_oracle():
    sd = W.h2p_1d()
    g = T.assemble_workload(sd)
    m = O.assemble(sd.breaks, sd.order, sd.nq, sd.minv, sd.V, sd.dV)
    ev_ref, vec = O.eig_banded(m["H0"], m["S"], 2, -1.2)
    ev, _ = T.ground_state(g, 2)
    say("levels", ev, ev_ref)
    assert np.abs((np.asarray(ev) - ev_ref) / ev_ref).max() < 1e-12
    # the plan: two waves, 128 chunks
    b = T.batch_create([g])
    T.batch_split(b, [sd.nsteps], 1)
    assert T.batch_two_wave(b).tolist() == [1]
    assert T.batch_chunks(b).tolist() == [128]
    # 120 steps on the flat top of the pulse (after the one-cycle ramp)
    ns, n0 = 120, 2400
    E = np.ascontiguousarray(sd.E[n0: n0 + ns + 1])
    psi0 = vec[0].astype(np.complex128)
    ref, cref = O.propagate(m, psi0, E, sd.dt, ns)
    for prec, tol in ((T.FP64, 1e-10), (T.FP32_REFINED, 1e-5)):
        psi = torch.from_numpy(psi0.copy()).cuda()
        Et = torch.from_numpy(E.copy()).cuda()
        o = torch.zeros(3 * (ns + 1), dtype=torch.float64, device="cuda")
        T.propagate(g, psi, Et, sd.dt, ns, prec, T.OBS_ALL, o)
        T.system_status(g)
        got = o.cpu().numpy().reshape(-1, 3)
        errs = [rel(got[:, k], ref[:, k]) for k in range(3)]
        say("h2p", prec, errs)
        assert errs[0] < tol and errs[1] < tol
        if prec == T.FP64:
            assert errs[2] < tol
            assert rel(psi.cpu().numpy(), cref) < 1e-10
