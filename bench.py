"""Throughput benchmark: batched Crank-Nicolson propagation on one MI355X.

Workload: 1024 seeded soft-Coulomb systems of uneven size (N ~ U{500..4000},
B-spline order 6-8, 4-cycle sin^2 pulses with seeded amplitude and carrier,
dt = 0.05), all propagated over their whole pulse in one persistent launch.
One benchmark step = one full propagation of the whole batch (every system,
every time step, with the norm/dipole/acceleration series).

Prints one JSON line.  Metric: complex DOF-steps/s = sum_i N_i nsteps_i /
wall time of the propagate call (HIP events on the launch stream), for the
FP32-refined path (one refinement sweep per step); the FP64 path is timed
beside it and the dipole error of the FP32 path against the FP64 path is
reported.  roofline.achieved = algorithmic bytes of the launch / its time;
roofline.traffic = HBM bytes of the launch measured with hardware counters.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "complex DOF-steps/s per GPU, FP32-refined vs FP64 at dipole error ≤1e-5"
HBM_PEAK_GBS = 8000.0
# device copy launched before the timed region: the calibration kernel of the
# HBM byte counters (FETCH_SIZE / WRITE_SIZE read this many bytes each way)
CALIB_COPY_BYTES = 512 * 2 ** 20
# HBM bytes of one FP32 batch call on this workload (the two-wave and the
# one-wave launch together), from two rocprofv3 --pmc runs of this script
# (FETCH_SIZE, then WRITE_SIZE) scaled by the copy calibration; valid only for
# the kernel sources they were taken on (sha256 of the listed files) and the
# default --split.  See profiles/propagate_kernel_fp32_batch1024_pmc.md.
TRAFFIC = {"sources_sha256": "9eb646a9691b338a6b3aba610fa68778d901ce4b2927dd343bdae9a04bad4ed0",
           "bytes_per_launch": 2.3280e+13, "split": 160}
# HBM bytes of one FP32 3D operator launch (apply3_kernel<3, float>, 97^3), from the
# two counter runs of profiles/apply3_kernel_hydrogen97_3d.md, for the sources listed.
TRAFFIC_3D = {"sources_sha256": "deb6768397d69cc4e21a03da513a5eaf98edeb3f80c55a2cb94f35dd38adeec0",
              "bytes_per_launch": 1.5981e+09}
KERNEL_SOURCES_3D = ["paper_2608_18472_amd/csrc/tdsez_3d.hip", "paper_2608_18472_amd/csrc/tdsez_krylov.hpp",
                     "paper_2608_18472_amd/csrc/tdsez_internal.hpp"]
KERNEL_SOURCES = ["paper_2608_18472_amd/csrc/tdsez_passes.hpp", "paper_2608_18472_amd/csrc/tdsez_propagate.hip",
                  "paper_2608_18472_amd/csrc/tdsez_internal.hpp", "paper_2608_18472_amd/csrc/tdsez_run.hpp",
                  "paper_2608_18472_amd/csrc/tdsez_prop_f32.hip"]
# Algorithmic bytes of one tensor-product operator application per unknown:
# the stored half of the potential stencil plus the input and output
# vectors (complex).  2D, order 6: 61 stored offsets.
STENCIL2D_BYTES = {4: 61 * 4 + 2 * 8, 8: 61 * 8 + 2 * 16}


def stencil3d_bytes(p, real_bytes):
    """3D: ((2p+1)^3 + 1) / 2 stored offsets (172 for cubic splines)."""
    w = 2 * p + 1
    return (w ** 3 + 1) // 2 * real_bytes + 2 * 2 * real_bytes


# The paper's Table II: 912 673 unknowns x 100 steps in 48.4 s on 256 Zen 4 cores.
TABLE2_DOFSTEPS_256 = 912673 * 100 / 48.4


def kernel_sources_sha(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if files is None else files):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def algorithmic_bytes(order, real_bytes, cplx_bytes):
    """Per DOF-step: the S, H0, D, G half bands (p+1 diagonals each) read
    once, the state read once and written once."""
    return 4 * order * real_bytes + 2 * cplx_bytes


def greville_gaussian(sd, width=1.0):
    """Initial state: B-spline coefficients of exp(-x^2/(2 w^2)) by quasi-
    interpolation at the Greville abscissae (unknown i is B-spline i+1)."""
    p = sd.order - 1
    br = sd.breaks
    t = np.r_[[br[0]] * p, br, [br[-1]] * p]
    N = sd.ndof
    g = np.arange(1, N + 1)
    xi = np.array([t[j + 1: j + 1 + p].mean() for j in g])
    return np.exp(-0.5 * (xi / width) ** 2).astype(np.complex128)


def _oracle_worker(args):
    idx, nsteps = args
    from oracle import oracle as O
    from paper_2608_18472_amd import workloads as W
    sd = W.config3(nsys=idx + 1, seed=0)[idx]
    m = O.assemble(sd.breaks, sd.order, sd.nq, None, sd.V, sd.dV)
    psi0 = greville_gaussian(sd)
    t0 = time.perf_counter()
    O.propagate(m, psi0, sd.E, sd.dt, nsteps)
    return sd.ndof * nsteps, time.perf_counter() - t0


def host_info():
    """Host core count and CPU model (the oracle's timing context)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"nproc": affinity, "cpu_count": os.cpu_count(), "cpu_model": model}


# worker processes of the oracle baseline: one per host core, at most 16
# (the share of host cores that goes with one GPU)
MAX_WORKERS = 16


def cpu_baseline(nsys_sample, nsteps):
    """The oracle (serial FP64 C) on a bounded sample of the batch: one
    system per worker process, one worker per host core (at most
    MAX_WORKERS).  The rate is DOF-steps of the sample per wall second; as a
    per-DOF-step rate it stands for the whole batch (extrapolated, not run)."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build()
    info = host_info()
    cores = min(MAX_WORKERS, info["nproc"] or 1)
    jobs = [(i, nsteps) for i in range(nsys_sample)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    dofsteps = sum(r[0] for r in res)
    out = {"value": dofsteps / wall, "unit": "DOF-steps/s", "cores": cores, "kind": "oracle",
           "sample": "first %d systems of the batch, %d steps each (%.3g DOF-steps), serial FP64 C, one system "
                     "per worker process on %d workers, wall %.1f s; the per-DOF-step rate is extrapolated to the "
                     "full batch, not run on it" % (nsys_sample, nsteps, dofsteps, cores, wall)}
    out.update(info)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsys", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-systems", type=int, default=96)
    ap.add_argument("--cpu-steps", type=int, default=6000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--tune-ms", type=float, default=3000.0,
                    help="partition autotuner budget per precision (setup, untimed); 0 keeps the default rule")
    ap.add_argument("--adjoint-waves", type=int, choices=[1, 2], default=2,
                    help="adjoint: waves per system (2: every system on two waves)")
    ap.add_argument("--max-waves", type=int, choices=[2, 4], default=2,
                    help="batch1d: the most waves a --split system may run on (4: cyclic reduction of the "
                         "separator system for systems whose four-wave plan has more than 128 chunks)")
    ap.add_argument("--split", type=int, default=160,
                    help="run this many of the costliest systems on two waves each (setup, untimed; "
                         "160 of 1024 measured best, 0 = one wave per system)")
    ap.add_argument("--workload", choices=["batch1d", "2d", "3d", "h2p", "adjoint"], default="batch1d",
                    help="batch1d: the batched 1D benchmark (default); 2d: a segment of the 512 x 512 "
                         "tensor-product workload; h2p: the 1D H2+ model (30 007 splines, one long "
                         "chain) over its whole pulse; adjoint: the pulse gradient of 64 double quantum "
                         "wells (N 1500, 20 000 steps, 64 amplitudes); 3d: hydrogen on 97^3 cubic "
                         "splines, 100 steps (the paper's strong-scaling workload)")
    ap.add_argument("--steps-2d", type=int, default=400, help="time steps of the 2D segment")
    ap.add_argument("--steps-3d", type=int, default=100,
                    help="time steps of the 3D workload (100 in the paper's strong-scaling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the propagation runs on a single device "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "2d":
        run_2d(args)
        return
    if args.workload == "h2p":
        run_h2p(args)
        return
    if args.workload == "3d":
        run_3d(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return

    import torch
    from paper_2608_18472_amd import tdsez as T
    from paper_2608_18472_amd import workloads as W

    torch.cuda.set_device(0)
    dev = "cuda"
    t_setup = time.perf_counter()
    defs = W.config3(nsys=args.nsys, seed=0)
    systems = [T.assemble_workload(s) for s in defs]
    batch = T.batch_create(systems)
    T.batch_set(batch, "refine", 1)
    psi_init, po, E, eo, obs, oo = T.pack_batch_inputs(defs, [np.zeros(s.ndof) for s in defs], dev)
    # initial states: every system's ground state (batched FP64 shift-and-invert on the GPU)
    t_gs = time.perf_counter()
    eps0 = T.ground_state_batched(batch, psi_init, po)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t_gs
    dts = [s.dt for s in defs]
    nsteps = [s.nsteps for s in defs]
    dofsteps = float(sum(s.ndof * s.nsteps for s in defs))
    if args.max_waves != 2:
        T.batch_set(batch, "max_waves", args.max_waves)
    if args.split > 0:
        T.batch_split(batch, nsteps, args.split)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    stream = torch.cuda.current_stream()
    # calibration copy for the HBM byte counters (outside every timed region)
    src = torch.empty(CALIB_COPY_BYTES // 8, dtype=torch.float64, device=dev)
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    def run(prec, k, obs_buf):
        psi = psi_init.clone()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(k):
            psi.copy_(psi_init)
            T.propagate_batched(batch, psi, po, E, eo, dts, nsteps, prec, T.OBS_ALL, obs_buf, oo, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        T.batch_status(batch, stream)
        return ev0.elapsed_time(ev1) / 1000.0, psi

    results = {}
    precs = [("fp32-refined", T.FP32_REFINED)] + ([] if args.no_fp64 else [("fp64", T.FP64)])
    obs_by = {}
    rule_chunks = T.batch_chunks(batch).copy()
    tuned = {}
    for name, prec in precs:
        if args.tune_ms > 0:
            # setup: per-system partition counts from short probe launches
            t_tune = time.perf_counter()
            ch = T.autotune(batch, prec, args.tune_ms)
            tuned[name] = {"seconds": time.perf_counter() - t_tune,
                           "systems_changed": int(np.sum(ch != rule_chunks))}
        ob = torch.zeros_like(obs)
        if args.warmup > 0:
            run(prec, args.warmup, ob)
        sec, psi = run(prec, args.steps, ob)
        results[name] = sec / args.steps
        obs_by[name] = ob.cpu().numpy()

    ms32 = results["fp32-refined"] * 1000.0
    value = dofsteps / results["fp32-refined"]
    eps_d = None
    eps_s = None
    if "fp64" in obs_by:
        from paper_2608_18472_amd import spectrum as SP
        e, es = [], []
        for i in range(len(defs)):
            a = obs_by["fp32-refined"][3 * eo[i]: 3 * eo[i] + 3 * (nsteps[i] + 1)].reshape(-1, 3)[:, 1]
            b = obs_by["fp64"][3 * eo[i]: 3 * eo[i] + 3 * (nsteps[i] + 1)].reshape(-1, 3)[:, 1]
            e.append(np.linalg.norm(a - b) / np.linalg.norm(b))
            qc = SP.cutoff_order(-eps0[i], defs[i].meta["E0"], defs[i].meta["omega"])
            es.append(SP.plateau_error(a, b, defs[i].dt, defs[i].meta["omega"], qc))
        eps_d = float(max(e))
        eps_s = float(max(es))
    # algorithmic bytes of one launch (FP32: 4-byte reals, 8-byte complex)
    alg_bytes = sum(s.ndof * s.nsteps * algorithmic_bytes(s.order, 4, 8) for s in defs)
    achieved = alg_bytes / results["fp32-refined"] / 1e9
    traffic = None
    if (TRAFFIC["bytes_per_launch"] is not None and TRAFFIC["sources_sha256"] == kernel_sources_sha()
            and TRAFFIC["split"] == args.split):
        traffic = TRAFFIC["bytes_per_launch"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched 1D soft-Coulomb propagation: %d systems, N~U{500..4000}, B-spline order "
                        "6-8, 4-cycle sin^2 pulses (E0 log-U[0.02,0.1], w U[0.03,0.08]), dt 0.05, seed 0"
                        % len(defs),
            "systems": len(defs),
            "dof_steps": dofsteps,
            "precision": "FP32 bands/factorisation/solve, FP64 residual/state/reductions",
            "fp64_value": dofsteps / results["fp64"] if "fp64" in results else None,
            "fp64_ms_per_step": results["fp64"] * 1000.0 if "fp64" in results else None,
            "dipole_rel_err_fp32_vs_fp64": eps_d,
            "spectrum_err_fp32_vs_fp64_dex": eps_s,
            "spectrum_metric": "max over systems and odd harmonics 3..q_cut+6 of |log10 S_fp32 - log10 S_fp64|, "
                               "S = w^4 |FT[d W]|^2, Kaiser window beta 8, q_cut = (Ip + 3.17 Up)/w",
            "refine_sweeps": 1,
            "two_wave_systems": int((T.batch_waves(batch) == 2).sum()),
            "four_wave_systems": int((T.batch_waves(batch) == 4).sum()),
            "autotune": tuned if tuned else None,
            "algorithmic_bytes_per_launch": alg_bytes,
            "setup_s": t_setup,
            "ground_state_s": t_gs,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
        },
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_systems, args.cpu_steps)
    print(json.dumps(line), flush=True)


def run_2d(args):
    """A segment of the 2D soft-Coulomb workload (512 x 512 order-6 splines on
    [-120, 120]^2, x-polarised sin^2 pulse E0 0.05, w 0.057, 4 cycles, dt
    0.05): steps 2000 .. 2000 + steps_2d of the pulse (field on), FP64 COCG
    and FP32-refined, both to relative residual 1e-12 per step."""
    import torch
    from paper_2608_18472_amd import tdsez as T
    from paper_2608_18472_amd import workloads as W

    torch.cuda.set_device(0)
    sd = W.config4()
    g = T.assemble_workload_2d(sd, with_force=False)  # norm and dipole only
    # initial state: product of the per-axis 1D ground states (library eigensolver)
    vecs = []
    for br in (sd.breaks_x, sd.breaks_y):
        xq = T.quad_points(br, sd.nq)
        s1 = T.assemble(br, sd.order, sd.nq, None, -1.0 / np.sqrt(xq * xq + 1.0), 0.0 * xq)
        ev, vec = T.ground_state(s1)
        vecs.append(vec[0])
    psi0 = torch.from_numpy(np.outer(vecs[1], vecs[0]).astype(np.complex128).reshape(-1)).cuda()
    # calibration copy for the HBM byte counters (outside the timed region)
    src = torch.empty(CALIB_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    n0, ns = 2000, args.steps_2d
    E = torch.from_numpy(np.ascontiguousarray(sd.E[n0: n0 + ns + 1])).cuda()
    stream = torch.cuda.current_stream()
    out = {}
    for name, prec in (("fp32-refined", T.FP32_REFINED), ("fp64", T.FP64)):
        o = torch.zeros(3 * (ns + 1), dtype=torch.float64, device="cuda")
        T.propagate_2d(g, psi0.clone(), E[:4].contiguous(), sd.dt, 3, prec, 3, o[:12], tol=1e-12)  # warm-up
        T.system2d_stats(g)
        psi = psi0.clone()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        T.propagate_2d(g, psi, E, sd.dt, ns, prec, 3, o, tol=1e-12, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1000.0
        steps, its, mx, sweeps = T.system2d_stats(g)
        out[name] = {"sec": sec, "its": its / steps, "sweeps": sweeps / steps, "obs": o.cpu().numpy()}
    d64 = out["fp64"]["obs"].reshape(-1, 3)[:, 1]
    d32 = out["fp32-refined"]["obs"].reshape(-1, 3)[:, 1]
    n = g.Nx * g.Ny
    # the operator kernel (dominant): algorithmic bytes per launch over its
    # event-timed average launch, FP32 as in the inner iterations
    ms32 = T.time_apply(g, T.FP32_REFINED, 50, stream)
    ms64 = T.time_apply(g, T.FP64, 50, stream)
    b32, b64 = n * STENCIL2D_BYTES[4], n * STENCIL2D_BYTES[8]
    # floor: two operator applications per step at HBM peak (per precision)
    floor = lambda b, sec: (2 * b / (HBM_PEAK_GBS * 1e9)) / (sec / ns)
    cpu = None if args.no_cpu else cpu_baseline_2d(60)
    line = {
        "metric": "complex DOF-steps/s per GPU (2D tensor-product segment)",
        "value": n * ns / out["fp32-refined"]["sec"],
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": ns,
        "warmup": 3,
        "ms_per_step": 1000.0 * out["fp32-refined"]["sec"] / ns,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "2D soft-Coulomb, 512 x 512 order-6 splines on [-120,120]^2, x-polarised sin^2 pulse "
                        "E0 0.05 w 0.057 4 cycles, dt 0.05, steps %d..%d, residual 1e-12" % (n0, n0 + ns),
            "fp32_refined": {"ms_per_step": 1000.0 * out["fp32-refined"]["sec"] / ns,
                             "inner_iterations_per_step": out["fp32-refined"]["its"],
                             "sweeps_per_step": out["fp32-refined"]["sweeps"]},
            "fp64": {"value": n * ns / out["fp64"]["sec"], "ms_per_step": 1000.0 * out["fp64"]["sec"] / ns,
                     "iterations_per_step": out["fp64"]["its"]},
            "dipole_rel_err_fp32_vs_fp64": float(np.linalg.norm(d32 - d64) / np.linalg.norm(d64)),
            "floor_fraction_fp32_refined": floor(b32, out["fp32-refined"]["sec"]),
            "floor_fraction_fp64": floor(b64, out["fp64"]["sec"]),
            "operator_kernel_ms": {"fp32": ms32, "fp64": ms64},
        },
        "roofline": {"bound": "hbm", "achieved": b32 / (ms32 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "apply_kernel<5, float> (FP32 operator of the inner iterations), %d B/unknown"
                               % STENCIL2D_BYTES[4]},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def run_3d(args):
    """The strong-scaling workload of the paper's Table II: hydrogen on 97^3
    cubic splines (hydrogenic knots on [-25, 25]^3, 912 673 unknowns, 343
    couplings per row), 100 Crank-Nicolson steps of 0.01 under the 800 nm
    field E0 sin(w t) (E0 0.053, w 0.057), relative residual 1e-12 per step
    (the paper's solver tolerance); FP32-refined and FP64."""
    import torch
    from paper_2608_18472_amd import tdsez as T
    from paper_2608_18472_amd import workloads as W

    torch.cuda.set_device(0)
    sd = W.hydrogen_3d(nsteps=args.steps_3d)
    t0 = time.perf_counter()
    g = T.assemble_workload_3d(sd)
    t_asm = time.perf_counter() - t0
    # initial state: the grid's ground state (the paper's eigensolve phase;
    # library shifted inverse iteration)
    t0 = time.perf_counter()
    e0, psi0 = T.ground_state_3d(g, -0.6, tol=1e-12)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t0
    ns = sd.nsteps
    E = torch.from_numpy(np.ascontiguousarray(sd.E[: ns + 1])).cuda()
    stream = torch.cuda.current_stream()
    # calibration copy for the HBM byte counters (outside the timed region)
    src = torch.empty(CALIB_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    out = {}
    for name, prec in (("fp32-refined", T.FP32_REFINED), ("fp64", T.FP64)):
        o = torch.zeros(3 * (ns + 1), dtype=torch.float64, device="cuda")
        T.propagate_3d(g, psi0.clone(), E[:4].contiguous(), sd.dt, 3, prec, 3, o[:12], tol=1e-12)  # warm-up
        T.system3d_stats(g)
        psi = psi0.clone()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        T.propagate_3d(g, psi, E, sd.dt, ns, prec, 3, o, tol=1e-12, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1000.0
        steps, its, mx, sweeps = T.system3d_stats(g)
        out[name] = {"sec": sec, "its": its / steps, "sweeps": sweeps / steps, "obs": o.cpu().numpy()}
    d64 = out["fp64"]["obs"].reshape(-1, 3)[:, 1]
    d32 = out["fp32-refined"]["obs"].reshape(-1, 3)[:, 1]
    n = g.N
    ms32 = T.time_apply(g, T.FP32_REFINED, 20, stream)
    ms64 = T.time_apply(g, T.FP64, 20, stream)
    b32, b64 = n * stencil3d_bytes(g.p, 4), n * stencil3d_bytes(g.p, 8)
    floor = lambda b, sec: (2 * b / (HBM_PEAK_GBS * 1e9)) / (sec / ns)
    cpu = None if args.no_cpu else cpu_baseline_3d()
    sec = out["fp32-refined"]["sec"]
    line = {
        "metric": "complex DOF-steps/s per GPU (3D hydrogen, the paper's strong-scaling workload)",
        "value": n * ns / sec,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": ns,
        "warmup": 3,
        "ms_per_step": 1000.0 * sec / ns,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": n * ns / sec / TABLE2_DOFSTEPS_256,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "3D hydrogen -1/r, 97^3 cubic splines (hydrogenic knots r1 0.125, 24 linear + 24 "
                        "exponential spans a side on [-25,25]), nq 6, %d steps dt 0.01 from the ground state, x field "
                        "0.053 sin(0.057 t), residual 1e-12" % ns,
            "unknowns": n,
            "assembly_s": t_asm,
            "ground_state_s": t_gs,
            "ground_state_energy": e0,
            "fp32_refined": {"ms_per_step": 1000.0 * sec / ns, "inner_iterations_per_step": out["fp32-refined"]["its"],
                             "sweeps_per_step": out["fp32-refined"]["sweeps"],
                             "floor_fraction": floor(b32, sec)},
            "fp64": {"value": n * ns / out["fp64"]["sec"], "ms_per_step": 1000.0 * out["fp64"]["sec"] / ns,
                     "iterations_per_step": out["fp64"]["its"], "floor_fraction": floor(b64, out["fp64"]["sec"])},
            "dipole_rel_err_fp32_vs_fp64": float(np.linalg.norm(d32 - d64) / np.linalg.norm(d64)),
            "operator_kernel_ms": {"fp32": ms32, "fp64": ms64},
            "vs_baseline_reference": "Table II: 48.4 s for the 100 steps on 256 Zen 4 cores (1.89e6 DOF-steps/s; "
                                     "assembly 10.9 s, eigensolve 15.0 s); another machine, context",
        },
        "roofline": {"bound": "hbm", "achieved": b32 / (ms32 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": (TRAFFIC_3D["bytes_per_launch"]
                                 if kernel_sources_sha(KERNEL_SOURCES_3D) == TRAFFIC_3D["sources_sha256"]
                                 and n == 912673 else None),
                     "kernel": "apply3_kernel<3, float> (FP32 operator of the inner iterations), %d B/unknown"
                               % stencil3d_bytes(g.p, 4)},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def cpu_baseline_3d(nsteps=1):
    """The oracle's 3D propagation (C operator over the 343-point rows,
    NumPy preconditioner transforms, COCG to 1e-12) on the full 97^3
    workload for `nsteps` steps (its assembly untimed)."""
    from oracle import oracle as O
    from paper_2608_18472_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        cores = 1
    # nq 4 instead of the workload's 6 keeps the oracle's assembly short; the
    # stencil, and so the cost of a step, does not depend on it
    sd = W.hydrogen_3d(nsteps=nsteps, nq=4)
    m3 = O.assemble_3d(sd.breaks_x, sd.breaks_y, sd.breaks_z, sd.order, sd.nq, sd.V)
    Nz, Ny, Nx = sd.shape
    g = [np.exp(-0.5 * np.linspace(-4, 4, k) ** 2) for k in (Nz, Ny, Nx)]
    psi0 = np.einsum("z,y,x->zyx", *g).astype(np.complex128)
    t0 = time.perf_counter()
    O.propagate_3d(m3, psi0, sd.E, sd.dt, nsteps, tol=1e-12)
    wall = time.perf_counter() - t0
    dof = Nx * Ny * Nz * nsteps
    out = {"value": dof / wall, "unit": "DOF-steps/s", "cores": cores, "kind": "oracle",
           "sample": "%d step(s) of the full 97^3 workload (%.3g DOF-steps; potential assembled with nq 4), serial C "
                     "operator with NumPy/BLAS preconditioner transforms, wall %.1f s (assembly untimed)"
                     % (nsteps, dof, wall)}
    out.update(host_info())
    return out


def run_h2p(args):
    """One long chain: the 1D H2+ model (N = 30 007, p = 7) over its whole
    6-cycle trapezoidal pulse (13 228 steps), FP32-refined then FP64, through
    the single-system call, whose plan spreads the chain over several
    workgroups (64 chunks of about 16 rows each, one grid-wide exchange of
    the workgroups' last separator blocks per solve)."""
    import torch
    from paper_2608_18472_amd import tdsez as T
    from paper_2608_18472_amd import workloads as W

    torch.cuda.set_device(0)
    sd = W.h2p_1d()
    g = T.assemble_workload(sd)
    ev, vec = T.ground_state(g, 2)
    psi0 = torch.from_numpy(vec[0].astype(np.complex128)).cuda()
    E = torch.from_numpy(np.ascontiguousarray(sd.E[: sd.nsteps + 1])).cuda()
    stream = torch.cuda.current_stream()
    ns = sd.nsteps
    out = {}
    for name, prec in (("fp32-refined", T.FP32_REFINED), ("fp64", T.FP64)):
        o = torch.zeros(3 * (ns + 1), dtype=torch.float64, device="cuda")
        T.propagate(g, psi0.clone(), E, sd.dt, 20, prec, T.OBS_ALL, o, stream)  # warm-up
        psi = psi0.clone()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        T.propagate(g, psi, E, sd.dt, ns, prec, T.OBS_ALL, o, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        T.system_status(g)
        out[name] = {"sec": ev0.elapsed_time(ev1) / 1000.0, "obs": o.cpu().numpy().reshape(-1, 3)}
    d64 = out["fp64"]["obs"][:, 1]
    d32 = out["fp32-refined"]["obs"][:, 1]
    n = sd.ndof
    sec = out["fp32-refined"]["sec"]
    alg = n * ns * algorithmic_bytes(sd.order, 4, 8)
    cpu = None if args.no_cpu else cpu_baseline_h2p(400)
    line = {
        "metric": "complex DOF-steps/s per GPU (1D H2+ model, one long chain)",
        "value": n * ns / sec,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": ns,
        "warmup": 20,
        "ms_per_step": 1000.0 * sec / ns,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "1D H2+ (R 2, soft-core eps 1.472), 30 007 degree-7 splines on [-4000,4000], mirrored "
                        "hydrogenic knots, 6-cycle trapezoidal pulse w 0.057 E0 0.0534, dt 0.05, whole pulse",
            "levels": [float(ev[0]), float(ev[1])],
            "workgroups_and_chunks": list(T.system_workgroups(g)),
            "fp64_value": n * ns / out["fp64"]["sec"],
            "fp64_ms_per_step": 1000.0 * out["fp64"]["sec"] / ns,
            "dipole_rel_err_fp32_vs_fp64": float(np.linalg.norm(d32 - d64) / np.linalg.norm(d64)),
            "final_norm_fp64": float(out["fp64"]["obs"][-1, 0]),
        },
        "roofline": {"bound": "hbm", "achieved": alg / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / sec / 1e9 / HBM_PEAK_GBS, "traffic": None},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def run_adjoint(args):
    """The pulse-gradient workload: 64 double quantum wells (N 1500, order 8,
    20 000 steps, config-2 geometry) driven by 64-amplitude Fourier pulses;
    one gradient = the differentiable forward series (one persistent
    propagation launch, FP64) and its backward (the discrete-adjoint launch
    with sqrt(Nt) checkpoints; each adjoint step substitutes with the
    factorisation kept by its segment's recomputation).  Metric: gradient
    DOF-steps/s = sum N nsteps
    / (forward + adjoint time); roofline of the adjoint launch with
    3 (3 (p+1) 8 + 2 16) = 672 algorithmic bytes per DOF-step (the
    checkpointing forward sweep, the segment recomputation and the adjoint
    step, each reading the S, H0, D bands and a state in and out)."""
    import torch
    from paper_2608_18472_amd import tdsez as T
    from paper_2608_18472_amd import workloads as W

    torch.cuda.set_device(0)
    defs, thetas, basis = W.config5()
    omega = defs[0].meta["omega"]
    gs = [T.assemble_workload(s) for s in defs]
    b = T.batch_create(gs)
    psi, po, E, eo, obs, oo = T.pack_batch_inputs(defs, [np.zeros(s.ndof) for s in defs])
    # every system's ground state in one launch (two-vector subspace
    # iteration: the double well's lowest doublet is split by 6e-5 Ha)
    T.ground_state_batched(b, psi, po, tol=1e-12, maxit=2000)
    if args.adjoint_waves == 2:
        # every system on two waves (N = 1500: 71 chunks), forward and adjoint
        T.batch_split(b, [s.nsteps for s in defs], len(defs))
    Bt = torch.from_numpy(basis).cuda()
    dt = [s.dt for s in defs]
    ns = [s.nsteps for s in defs]
    mask = T.OBS_NORM | T.OBS_DIPOLE
    stream = torch.cuda.current_stream()
    dofsteps = float(sum(s.ndof * s.nsteps for s in defs))

    def gradient():
        th = torch.from_numpy(thetas.copy()).cuda().requires_grad_(True)
        Ep = torch.cat([Bt @ th[i] for i in range(len(defs))])
        ev0, ev1, ev2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        ev0.record(stream)
        ser = T.observable_series(Ep, b, psi, po, eo, dt, ns, oo, mask)
        ev1.record(stream)
        J = 0.0
        for i in range(len(defs)):
            d = ser[oo[i]: oo[i] + 3 * (ns[i] + 1)].reshape(-1, 3)[:, 1]
            J = J + W.harmonic_yield(d, dt[i], omega)
        J.backward()
        ev2.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3, ev1.elapsed_time(ev2) / 1e3, th.grad

    for _ in range(max(args.warmup, 1)):
        gradient()
    # the adjoint launch alone, timed with events on its stream, from the
    # series' gradient of the last evaluation
    ser = torch.zeros_like(obs)
    psi_w = psi.clone()
    Ep = torch.cat([Bt @ torch.from_numpy(thetas[i]).cuda() for i in range(len(defs))])
    T.propagate_batched(b, psi_w, po, Ep, eo, dt, ns, T.FP64, mask, ser, oo)
    T.batch_status(b)
    sr = ser.clone().requires_grad_(True)
    J = 0.0
    for i in range(len(defs)):
        d = sr[oo[i]: oo[i] + 3 * (ns[i] + 1)].reshape(-1, 3)[:, 1]
        J = J + W.harmonic_yield(d, dt[i], omega)
    J.backward()
    dJ = sr.grad.contiguous()
    gE = torch.zeros_like(Ep)
    ta = []
    for _ in range(max(args.steps, 1)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        T.adjoint_batched(b, psi, po, Ep, eo, dt, ns, mask, dJ, oo, gE, None, 0, T.FP64, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        T.batch_status(b)
        ta.append(e0.elapsed_time(e1) / 1e3)
    t_adj = float(np.mean(ta))
    tf, tb = [], []
    for _ in range(max(args.steps, 1)):
        f, bk, g = gradient()
        tf.append(f)
        tb.append(bk)
    t_f, t_b = float(np.mean(tf)), float(np.mean(tb))
    alg = dofsteps * 3 * (3 * 8 * 8 + 2 * 16)
    cpu = None if args.no_cpu else cpu_baseline_adjoint(2000)
    line = {
        "metric": "gradient DOF-steps/s per GPU (discrete adjoint of the pulse-gradient workload, FP64)",
        "value": dofsteps / (t_f + t_b),
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": max(args.steps, 1),
        "warmup": max(args.warmup, 1),
        "ms_per_step": 1000.0 * (t_f + t_b),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "64 GaAs/AlGaAs double quantum wells (10 nm wells, 4 nm barrier, N 1500, order 8), "
                        "Fourier pulses with 64 amplitudes (8-cycle 0.3 eV sin^2 fit + 10% seeded noise), "
                        "20000 steps, J = harmonic yield of orders 15-35, sqrt(Nt) checkpoints",
            "systems": len(defs),
            "waves_per_system": args.adjoint_waves,
            "dof_steps": dofsteps,
            "forward_s": t_f,
            "backward_s": t_b,
            "adjoint_launch_s": t_adj,
            "algorithmic_bytes_adjoint_launch": alg,
        },
        "roofline": {"bound": "hbm", "achieved": alg / t_adj / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / t_adj / 1e9 / HBM_PEAK_GBS, "traffic": None},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def cpu_baseline_adjoint(nsteps):
    """The oracle's FP64 adjoint (forward storing every state, then the
    reverse sweep) on one system of the workload for its first nsteps steps,
    one core; DOF-steps of the gradient per second."""
    from oracle import oracle as O
    from paper_2608_18472_amd import workloads as W
    O.build()
    defs, thetas, basis = W.config5(nsys=1)
    sd = defs[0]
    m = O.assemble(sd.breaks, sd.order, sd.nq, sd.minv, sd.V, sd.dV)
    xq, _ = O.quad_points(sd.breaks, sd.nq)
    vmin = float(np.min(sd.V(xq)))
    ev, vec = O.eig_banded(m["H0"], m["S"], 2, vmin - 1e-3 * (abs(vmin) + 1.0))
    rng = np.random.default_rng(0)
    dJ = np.zeros((nsteps + 1, 3))
    dJ[:, 1] = rng.normal(size=nsteps + 1)
    t0 = time.perf_counter()
    O.adjoint(m, vec[0].astype(np.complex128), sd.E, sd.dt, nsteps, dJ, with_accel=False)
    wall = time.perf_counter() - t0
    dof = sd.ndof * nsteps
    out = {"value": dof / wall, "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
           "sample": "oracle FP64 adjoint of one system, first %d steps (%.3g DOF-steps), one core, wall %.1f s; "
                     "per-DOF-step rate" % (nsteps, dof, wall)}
    out.update(host_info())
    return out


def cpu_baseline_h2p(nsteps):
    """The oracle (serial FP64 C, one core: a single system) on the first
    nsteps steps of the H2+ workload."""
    from oracle import oracle as O
    from paper_2608_18472_amd import workloads as W
    O.build()
    sd = W.h2p_1d()
    m = O.assemble(sd.breaks, sd.order, sd.nq, sd.minv, sd.V, sd.dV)
    ev, vec = O.eig_banded(m["H0"], m["S"], 1, -1.2)
    t0 = time.perf_counter()
    O.propagate(m, vec[0].astype(np.complex128), sd.E, sd.dt, nsteps)
    wall = time.perf_counter() - t0
    dof = sd.ndof * nsteps
    out = {"value": dof / wall, "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
           "sample": "first %d steps of the H2+ pulse (%.3g DOF-steps), serial FP64 C, wall %.1f s"
                     % (nsteps, dof, wall)}
    out.update(host_info())
    return out


def cpu_baseline_2d(nsteps):
    """The oracle's 2D propagation (C operator, NumPy/BLAS preconditioner
    transforms, COCG to 1e-12) on the 128 x 128 reduced grid of the same
    workload, field on; DOF-steps/s with the BLAS thread count as cores."""
    from oracle import oracle as O
    from paper_2608_18472_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        cores = 1
    sd = W.config4(n=128, nsteps=nsteps)
    m2 = O.assemble_2d(sd.breaks_x, sd.breaks_y, sd.order, sd.nq, sd.V)
    vx = np.exp(-0.5 * np.linspace(-4, 4, m2["Nx"]) ** 2)
    vy = np.exp(-0.5 * np.linspace(-4, 4, m2["Ny"]) ** 2)
    psi0 = np.outer(vy, vx).astype(np.complex128)
    E = 0.05 * np.sin(0.057 * sd.dt * np.arange(nsteps + 1) + 0.3)
    t0 = time.perf_counter()
    O.propagate_2d(m2, psi0, E, sd.dt, nsteps, tol=1e-12)
    wall = time.perf_counter() - t0
    dof = m2["Nx"] * m2["Ny"] * nsteps
    out = {"value": dof / wall, "unit": "DOF-steps/s", "cores": cores, "kind": "oracle",
           "sample": "128 x 128 reduced grid of the 2D workload, %d steps (%.3g DOF-steps), C operator with "
                     "NumPy/BLAS preconditioner transforms, wall %.1f s" % (nsteps, dof, wall)}
    out.update(host_info())
    return out


def _symband_mul(band, c):
    p1, N = band.shape
    y = band[0] * c
    for d in range(1, p1):
        y[:-d] += band[d, :N - d] * c[d:]
        y[d:] += band[d, :N - d] * c[:-d]
    return y


if __name__ == "__main__":
    main()
