"""The allocation-free entry point tdsez_propagate_noalloc against
tdsez_propagate (the same kernels and plan): two calls in a row, the second
with a smaller system, both precisions, one- and two-wave plans; the latched
status comes back through the caller's device buffer."""
import sys

import numpy as np
import pytest

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


def one(sd, ns, prec):
    g = T.assemble_workload(sd)
    ev, vec = T.ground_state(g, 1)
    psi0 = vec[0].astype(np.complex128)
    E = torch.from_numpy(np.ascontiguousarray(sd.E[: ns + 1], dtype=np.float64)).cuda()
    out = []
    for noalloc in (False, True):
        psi = torch.from_numpy(psi0.copy()).cuda()
        o = torch.zeros(3 * (ns + 1), dtype=torch.float64, device="cuda")
        if noalloc:
            st = torch.full((4,), -7, dtype=torch.int32, device="cuda")
            T.propagate_noalloc(g, psi, E, sd.dt, ns, prec, T.OBS_ALL, o, st)
            torch.cuda.synchronize()
            assert st[0].item() == 0
        else:
            T.propagate(g, psi, E, sd.dt, ns, prec, T.OBS_ALL, o)
            T.system_status(g)
        out.append((o.cpu().numpy(), psi.cpu().numpy()))
    return out


@pytest.mark.parametrize("prec,tol", [(T.FP64, 1e-10), (T.FP32_REFINED, 1e-5)])
def test_noalloc_matches_propagate_on_two_calls(prec, tol):
    # first call: a system on two waves (N 1500 > the one-wave plan),
    # second call: a smaller one-wave system (config 1, N 1004)
    ns = 150
    V, dV = W.soft_coulomb(2.0)
    E = 0.05 * np.sin(0.057 * 0.05 * np.arange(ns + 1) + 0.3)
    big = W.System("two-wave", W.breaks_uniform(200.0, 1500 - 8 + 3), 8, lambda x: np.ones_like(x), V, dV, 10, E,
                   0.05, ns, True)
    small = W.config1(nsteps=ns)
    small.E = E.copy()
    for sd in (big, small):
        (o_ref, c_ref), (o_na, c_na) = one(sd, ns, prec)
        e = max(rel(o_na[k::3], o_ref[k::3]) for k in range(3))
        say(sd.name, prec, "rel diff", e, "bitwise", bool(np.array_equal(o_na, o_ref)))
        assert e < tol * 1e-3
        assert rel(c_na, c_ref) < tol * 1e-3


def test_noalloc_latches_device_errors_into_the_callers_status():
    sd = W.config1(nsteps=20)
    g = T.assemble_workload(sd)
    psi0 = np.zeros(g.N, np.complex128)
    psi0[g.N // 2] = 1.0
    E = sd.E[:21].copy()
    E[5] = np.nan
    psi = torch.from_numpy(psi0).cuda()
    o = torch.zeros(63, dtype=torch.float64, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    T.propagate_noalloc(g, psi, torch.from_numpy(E).cuda(), sd.dt, 20, T.FP64, T.OBS_ALL, o, st)
    torch.cuda.synchronize()
    assert st[0].item() == 5  # ENONFINITE
    with pytest.raises(T.TdsezError) as e:
        T.propagate_noalloc(g, psi, torch.from_numpy(E).cuda(), 0.0, 20, T.FP64, T.OBS_ALL, o, st)
    assert e.value.status == 1
