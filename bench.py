"""Benchmark of the SLLBM stream + collide step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload riemann|svi|sod|tgv|adjoint_tgv]
                    [--precision fp32|fp64] [--path auto|direct|tiled|records]
                    [--no-fp64] [--no-svi] [--no-adjoint] [--no-cpu-baseline]

One "step" is one time step of the whole hot path over the grid: departure
gather with Lagrange interpolation, moments, temperature, 4th-order
equilibrium, BGK relaxation and store (one fused kernel launch), with inputs
resident in HBM.  Default workload: the four-quadrant Riemann problem on
512 x 512 cells of order 2 (1025^2 nodes, f and g populations, float32
populations with float64 moments).  Prints one JSON line; besides the headline
it carries the FP64 run of the same workload and the FP32-FP64 difference of
the moments after the timed steps, the stretched shock-vortex grid with
departure records and with per-axis tables, the adjoint/forward cost ratio of
the checkpointed Taylor-Green rollout, and the FP64 oracle timed on a sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q25 node-updates/s FP32 vs FP64 at stated error; adjoint/forward cost ratio"
HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_1910_13918_amd import workloads as W
    if name == "riemann":
        return W.riemann(512, 2), "riemann2d_512x512cells_p2"
    if name == "svi":
        return W.svi(1024, 512, 3), "shock_vortex_1024x512cells_p3_stretched"
    if name == "sod":
        return W.sod(1024, 4, 3), "sod_1024x4cells_p3"
    if name == "tgv":
        return W.tgv(), "tgv_8x8cells_p2"
    if name == "adjoint_tgv":
        return W.adjoint_tgv(), "tgv_128x128cells_p4"
    if name == "curvilinear":
        return W.tgv_wavy(256, 4, amp=0.3), "tgv_wavy_256x256cells_p4_amp0.3"
    raise SystemExit(f"unknown workload {name}")


def bytes_per_node_update(wl, precision, path):
    """Algorithmic HBM bytes per node update: every population read once and
    written once (tables excluded); per-(node, velocity) departure records add
    a 4-byte cell index and two reference coordinates per velocity."""
    size = 8 if precision == "fp64" else 4
    b = 2 * wl.nsets * 25 * size
    if path == "records":
        b += 25 * (4 + 2 * size)
    return b


def mfma_flops_per_node_update(wl):
    """Matrix-core flops of the x-pass per node update: per tile of 64 x 4
    nodes and x-component, 4 blocks of 16 columns x 16 (set, row) pairs x
    4 ks columns, 2 flops each, 5 components per phase, 5 phases."""
    ks = (16 + 2 * wl.p + 3) // 4
    return 5 * 5 * 4 * (16 * 16 * 4 * ks * 2) / (64 * 4)


def profiled_traffic(wname, precision, path):
    """HBM bytes per launch from the committed counter profile of this workload
    and kernel family (FETCH_SIZE and WRITE_SIZE scaled by a copy of known
    size), or None when no profile exists or the kernel source has changed
    since it was taken."""
    import hashlib
    tag = {"riemann2d_512x512cells_p2": "riemann512_p2",
           "shock_vortex_1024x512cells_p3_stretched": "svi1024x512_p3",
           "tgv_wavy_256x256cells_p4_amp0.3": "curvilinear_tgv_wavy256_p4",
           "tgv3d_64^3cells_p2": "d3q125_tgv3d64_p2"}.get(wname)
    if tag is None:
        return None
    f = os.path.join(ROOT, "profiles", f"stream_collide_{tag}_{precision}_{path}.json")
    if not os.path.exists(f):
        f = os.path.join(ROOT, "profiles", f"stream_collide_{tag}_{precision}.json")
    if not os.path.exists(f):
        return None
    prof = json.load(open(f))
    if prof.get("path") != path:
        return None
    m = hashlib.sha256()
    for src in prof["source_files"]:
        m.update(open(os.path.join(ROOT, src), "rb").read())
    if m.hexdigest()[:16] != prof["source_sha256_16"]:
        return None
    return prof["traffic_bytes_per_launch"]


def timed(wl, precision, path, steps, warmup):
    """Initialise the workload, run `warmup` steps, then time `steps` steps with
    HIP events on the solver's stream.  Returns (solver, ms, unstable flag)."""
    import torch

    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(wl, precision=precision, path=path)
    s.init_from_workload()
    # initial mass, for the drift reported after the run (untimed; axis-product
    # grids only)
    s.mass0 = s.mass() if wl.vertices is None else None
    s.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    s.step(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    unstable, _ = s.flags()
    return s, ev0.elapsed_time(ev1), unstable


def shock_vortex_entry(precision, steps=20, warmup=3):
    """Throughput on the stretched shock-vortex grid (1024 x 512 cells, p = 3,
    3073 x 1536 nodes, f + g, Pr = 0.75 as in the paper) with per-(node,
    velocity) departure records and with the per-axis tables the separable map
    allows; the last line repeats the per-axis tables at Pr = 1 (BGK only) to
    show the cost of the quasi-equilibrium term."""
    import copy
    wl, wname = workload("svi")
    wl1 = copy.copy(wl)
    wl1.Pr = 1.0
    out = {"workload": wname, "Pr": wl.Pr, "steps": steps, "warmup": warmup}
    for label, w, path in (("records", wl, "records"), ("axis_tables", wl, "auto"),
                           ("axis_tables_pr1", wl1, "auto")):
        s, ms, unstable = timed(w, precision, path, steps, warmup)
        nu_s = s.n * steps / (ms * 1e-3)
        bpn = bytes_per_node_update(wl, precision, s.resolved_path())
        out[label] = {"path": s.resolved_path(), "value": nu_s, "unit": "node-updates/s",
                      "ms_per_step": ms / steps, "bytes_per_node_update": bpn,
                      "achieved_gbs": nu_s * bpn / 1e9, "frac": nu_s * bpn / 1e9 / HBM_PEAK_GBS,
                      "unstable_flag": unstable}
        if label != "axis_tables_pr1":  # counters taken at Pr = 0.75
            tr = profiled_traffic(wname, precision, s.resolved_path())
            out[label]["traffic"] = tr
            out[label]["traffic_over_algorithmic"] = (tr / (s.n * bpn)) if tr else None
        s.close()
    return out


def curvilinear_entry(precision, steps=20, warmup=3):
    """Throughput on a curvilinear periodic mesh: the Taylor-Green vortex on
    256 x 256 bilinear cells of order 4 (1024^2 nodes, isothermal, cells
    distorted by the wavy map with amplitude 0.3), departure points located
    on the host, streamed by the records gather (FP32: 200 B of populations
    and 300 B of records per node update)."""
    from paper_1910_13918_amd import workloads as W
    wl = W.tgv_wavy(256, 4, amp=0.3)
    s, ms, unstable = timed(wl, precision, "auto", steps, warmup)
    nu_s = s.n * steps / (ms * 1e-3)
    bpn = bytes_per_node_update(wl, precision, s.resolved_path())
    tr = profiled_traffic("tgv_wavy_256x256cells_p4_amp0.3", precision, s.resolved_path())
    out = {"workload": "tgv_wavy_256x256cells_p4_amp0.3", "path": s.resolved_path(),
           "steps": steps, "warmup": warmup, "value": nu_s, "unit": "node-updates/s",
           "ms_per_step": ms / steps, "bytes_per_node_update": bpn,
           "achieved_gbs": nu_s * bpn / 1e9, "frac": nu_s * bpn / 1e9 / HBM_PEAK_GBS,
           "unstable_flag": unstable, "traffic": tr,
           "traffic_over_algorithmic": tr / (s.n * bpn) if tr else None}
    s.close()
    return out


def d3q125_entry(steps=20, warmup=3):
    """Throughput of the three-dimensional step (isothermal D3Q125): the 3-D
    Taylor-Green vortex on 64^3 cells of order 2 (128^3 nodes, 125 planes;
    float32: 1000 B per node update, every population read and written once),
    float32 and float64, with their moment differences after the run."""
    import numpy as np
    import torch

    from paper_1910_13918_amd import workloads as W
    from paper_1910_13918_amd.solver import Solver3D
    wl = W.tgv3d(64, 2)
    wname = "tgv3d_64^3cells_p2"
    out = {"workload": wname, "steps": steps, "warmup": warmup}
    mom = {}
    for precision in ("fp32", "fp64"):
        s = Solver3D.from_workload(wl, precision=precision)
        s.init_from_workload()
        s.step(warmup)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(s.stream)
        s.step(steps)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        nu_s = s.n * steps / (ms * 1e-3)
        bpn = 2 * 125 * (8 if precision == "fp64" else 4)
        path = "rows3d"
        tr = profiled_traffic(wname, precision, path)
        out[precision] = {"path": path, "value": nu_s, "unit": "node-updates/s",
                          "ms_per_step": ms / steps,
                          "bytes_per_node_update": bpn, "achieved_gbs": nu_s * bpn / 1e9,
                          "frac": nu_s * bpn / 1e9 / HBM_PEAK_GBS, "traffic": tr,
                          "traffic_over_algorithmic": tr / (s.n * bpn) if tr else None,
                          "unstable_flag": s.flags()[0]}
        mom[precision] = s.moments()
        out["nodes"] = s.n
        s.close()
    a, b = mom["fp32"], mom["fp64"]
    umax = max(np.abs(b[k]).max() for k in (1, 2, 3))
    out["fp32_vs_fp64_after_steps"] = {
        "rho_max_rel": float(np.abs(a[0] - b[0]).max() / np.abs(b[0]).max()),
        "u_max_rel": float(max(np.abs(a[k] - b[k]).max() for k in (1, 2, 3)) / umax)}
    return out


def aux_kernels(s, reps=20):
    """Average duration of the initialisation f = f_eq (from device fields),
    the moments output and the mass reduction on the benchmark grid, with
    their algorithmic bytes: init reads 4 float64 fields and writes every
    population; moments read every population and write 4 float64 fields;
    the mass reads the f populations (its call returns the value to the host,
    so its time includes the device-to-host copy and synchronisation)."""
    import torch

    from paper_1910_13918_amd import sllbm as C
    X, Y = s.coords()
    fields = [torch.tensor(a, device=s.device) for a in s.workload.fields(X, Y)]
    outs = [torch.empty(s.n, dtype=torch.float64, device=s.device) for _ in range(4)]
    size = 8 if s.precision == "fp64" else 4
    pops = s.nsets * 25 * size

    def timed_call(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        for _ in range(reps):
            fn()
        e1.record(s.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {}
    for name, fn, nbytes in (
            ("init_eq", lambda: C.sllbm_init_macro(s.ctx, *[t.data_ptr() for t in fields], 1),
             32 + pops),
            ("moments", lambda: C.sllbm_moments(s.ctx, *[t.data_ptr() for t in outs], 1), pops + 32),
            ("mass", lambda: C.sllbm_mass(s.ctx), 25 * size)):
        ms = timed_call(fn)
        res[name] = {"ms": ms, "bytes_per_node": nbytes, "achieved_gbs": s.n * nbytes / (ms * 1e6)}
    res["mass"]["includes_host_sync"] = True
    return res


def mfma_bf16_flops_per_node_update(wl):
    """Matrix-core flops of the bfloat16 x-pass per node update: per tile of
    64 x 4 nodes and x-component, 4 blocks of one 16 x 16 x 32 product, 5
    components per phase, 5 phases."""
    return 5 * 5 * 4 * (16 * 16 * 32 * 2) / (64 * 4)


def _moment_errors(got, ref):
    """max and L2 relative errors of rho, u (vector) and theta."""
    import numpy as np
    d_u = np.hypot(got[1] - ref[1], got[2] - ref[2])
    u_ref = np.hypot(ref[1], ref[2])
    out = {}
    for name, d, r in (("rho", got[0] - ref[0], ref[0]), ("u", d_u, u_ref),
                       ("T", got[3] - ref[3], ref[3])):
        out[name + "_max_rel"] = float(np.abs(d).max() / np.abs(r).max())
        out[name + "_l2_rel"] = float(np.linalg.norm(d) / np.linalg.norm(r))
    return out


def bf16_experiment(wl, steps, warmup, fp64_run):
    """The bfloat16 x-pass (SLLBM_BF16X) on the benchmark grid: throughput,
    HBM fraction and matrix-core rate, its moments after the same steps
    against the FP64 GPU run, and the seeded Riemann problem on 64 x 64 cells
    to t = 0.25 against the FP64 oracle's moments (committed golden written by
    the oracle alone).  Errors are reported, not bounded."""
    import numpy as np

    from paper_1910_13918_amd import workloads as W
    from paper_1910_13918_amd.solver import Solver
    sb, msb, unstable = timed(wl, "bf16x", "auto", steps, warmup)
    v = sb.n * steps / (msb * 1e-3)
    bpn = bytes_per_node_update(wl, "fp32", "mfma")
    flops = v * mfma_bf16_flops_per_node_update(wl)
    res = {"path": sb.resolved_path(), "value": v, "unit": "node-updates/s",
           "ms_per_step": msb / steps, "achieved_gbs": v * bpn / 1e9,
           "frac": v * bpn / 1e9 / HBM_PEAK_GBS, "mfma_tflops": flops / 1e12,
           "mfma_frac_of_bf16_dense_peak": flops / 2.5e15, "unstable_flag": unstable}
    if fp64_run is not None:
        m64, dm64 = fp64_run
        res["vs_fp64_gpu_after_steps"] = dict(_moment_errors(sb.moments(), m64),
                                             steps=steps + warmup,
                                             mass_rel_change=sb.mass() / sb.mass0 - 1.0,
                                             mass_rel_change_fp64=dm64)
    sb.close()
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "riemann64_reference.json")))
    nodes = np.array(ref["nodes"])
    want = [np.array(ref[k]) for k in ("rho", "ux", "uy", "T")]
    w64 = W.riemann(64, 2)
    s = Solver.from_workload(w64, precision="bf16x")
    s.init_from_workload()
    m0 = s.mass()
    s.step(w64.steps)
    got = [a[nodes] for a in s.moments()]
    res["riemann64_t0.25_vs_fp64_oracle"] = dict(_moment_errors(got, want), steps=w64.steps,
                                                 mass_rel_change=s.mass() / m0 - 1.0)
    s.close()
    return res


def adjoint_cost(precision="fp32", every=50, reps=3):
    """Forward and backward time of the checkpointed rollout on the adjoint
    workload (Taylor-Green, 128 x 128 cells, p = 4, 500 steps, loss = kinetic
    energy + misfit to a seeded target): backward includes the recomputation."""
    import numpy as np
    import torch

    from paper_1910_13918_amd import sllbm as C
    from paper_1910_13918_amd import workloads as W
    from paper_1910_13918_amd.adjoint import rollout
    from paper_1910_13918_amd.solver import Solver
    wl = W.adjoint_tgv()
    s = Solver.from_workload(wl, precision=precision)
    X, Y = s.coords()
    rho0, ux0, uy0, _ = wl.fields(X, Y)
    ut, vt = W.fourier_target(X, Y, wl.meta["U0"])
    mx, my = np.zeros(s.nx), np.zeros(s.ny)
    C.sllbm_mass_weights(s.ctx, mx.ctypes.data, my.ctypes.data)
    t = lambda a: torch.tensor(a, device="cuda")
    M, ut, vt = t(np.outer(my, mx).reshape(-1)), t(ut), t(vt)
    fwd, bwd = [], []
    for _ in range(reps + 1):
        u0 = t(ux0).requires_grad_(True)
        v0 = t(uy0).requires_grad_(True)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        rho, ux, uy = rollout(t(rho0), u0, v0, s, wl.steps, every)
        e1.record()
        L = 0.5 * (M * rho * (ux * ux + uy * uy)).sum() + (M * ((ux - ut) ** 2 + (uy - vt) ** 2)).sum()
        L.backward()
        e2.record()
        torch.cuda.synchronize()
        fwd.append(e0.elapsed_time(e1))
        bwd.append(e1.elapsed_time(e2))
    kern = adjoint_step_kernel(s)
    s.close()
    f, b = min(fwd[1:]), min(bwd[1:])
    return {"workload": "tgv_128x128cells_p4_500steps", "precision": precision,
            "checkpoint_every": every, "forward_ms": f, "backward_ms": b, "ratio": b / f,
            "adjoint_step_kernel": kern}


def adjoint_step_kernel(s, reps=50):
    """Average duration of one fused adjoint step (the transposed gather S^T
    fused with the previous step's collision Jacobian, sllbm_adjoint_step
    with a moments record) on the solver's grid, with its algorithmic bytes
    per node: mu read and lambda written (S 25 values each) plus the K
    recorded float64 moments read."""
    import torch

    from paper_1910_13918_amd import sllbm as C
    size = 4 if s.precision != "fp64" else 8
    K = s.recorded_moments
    s.init_from_workload()
    mom = s.step_record(1)[0].contiguous()
    mu = s.populations_device().contiguous()
    out = torch.empty_like(mu)
    C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), mom.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    for _ in range(reps):
        C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), mom.data_ptr(), out.data_ptr())
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bpn = 2 * s.nsets * 25 * size + 8 * K
    return {"ms": ms, "bytes_per_node": bpn, "nodes": s.n,
            "achieved_gbs": s.n * bpn / (ms * 1e6), "frac": s.n * bpn / (ms * 1e6) / HBM_PEAK_GBS}


# ---- CPU baseline: the FP64 oracle on the host's cores ---------------------------
_ORACLE = {}


def _oracle_setup(wname):
    """Oracle simulation and initial state of a bench workload (in a worker)."""
    from oracle.grid import Grid
    from oracle.sllbm import Sim
    wl, _ = workload(wname)
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)
    X, Y = g.coords()
    _ORACLE["sim"] = sim
    _ORACLE["F0"] = sim.init(*wl.fields(X, Y))


def _oracle_chunk(nodes):
    """One oracle step at `nodes` (worker side); returns the chunk's size."""
    _ORACLE["sim"].step(_ORACLE["F0"], nodes)
    return len(nodes)


def cpu_baseline(wname, solver_state, sample_nodes=250000, seed=0):
    """Time the FP64 oracle on the host: one full step of the workload (every
    node) split over worker processes on all host cores the box grants (at
    most 16), and one step at `sample_nodes` seeded nodes on one core, from
    the same initial state as the GPU.  The single-core sample also gives the
    GPU's one-step error at those nodes."""
    import multiprocessing as mp

    import numpy as np
    _oracle_setup(wname)
    sim, F0 = _ORACLE["sim"], _ORACLE["F0"]
    n_all = sim.grid.nnodes
    rng = np.random.default_rng(seed)
    nodes = np.sort(rng.choice(n_all, size=min(sample_nodes, n_all), replace=False))
    t0 = time.perf_counter()
    F1 = sim.step(F0, nodes)
    t1 = time.perf_counter() - t0
    err = float(np.abs(solver_state[:, :, nodes] - F1).max() / np.abs(F1).max())
    host_cores = os.cpu_count() or 1
    workers = max(1, min(host_cores, 16))
    # one thread per worker process (set before the workers import numpy)
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers, initializer=_oracle_setup,
                                          initargs=(wname,)) as pool:
            pool.map(_oracle_chunk, [np.arange(1)] * workers)  # every worker set up
            chunks = np.array_split(np.arange(n_all), 8 * workers)
            t0 = time.perf_counter()
            done = sum(pool.map(_oracle_chunk, chunks, chunksize=1))
            tw = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    assert done == n_all
    return {"value": n_all / tw, "unit": "node-updates/s", "cores": workers, "kind": "oracle",
            "host_cores": host_cores,
            "sample": f"one FP64 oracle step at all {n_all} nodes of the same workload over "
                      f"{workers} worker processes ({tw:.1f} s; numpy, one thread each)",
            "single_core": {"value": len(nodes) / t1, "unit": "node-updates/s", "cores": 1,
                            "sample": f"one step at {len(nodes)} seeded nodes ({t1:.1f} s)"}}, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="riemann")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--path", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost ratio")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-mfma", action="store_true", help="skip the matrix-core x-pass line")
    ap.add_argument("--no-svi", action="store_true",
                    help="skip the shock-vortex (stretched 1024 x 512 cells, p = 3) and "
                         "curvilinear-mesh lines")
    ap.add_argument("--d3q125-only", action="store_true",
                    help="only time the three-dimensional step (prints its JSON object)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the checkpointed adjoint rollout (prints its JSON object)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device-to-device three times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 3}))
        return
    if args.d3q125_only:
        print(json.dumps(d3q125_entry(args.steps, args.warmup)))
        return
    if args.adjoint_only:
        print(json.dumps(adjoint_cost(args.precision)))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the stream + collide step is a single-GPU kernel "
              "(the multi-GPU domain decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_1910_13918_amd.solver import Solver
    wl, wname = workload(args.workload)
    s, ms, unstable = timed(wl, args.precision, args.path, args.steps, args.warmup)
    s_path = s.resolved_path()
    nu_s = s.n * args.steps / (ms * 1e-3)
    bpn = bytes_per_node_update(wl, args.precision, s_path)
    achieved = nu_s * bpn / 1e9
    out = {
        "metric": METRIC, "value": nu_s, "unit": "node-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": wname, "nodes": s.n, "populations": wl.nsets * 25,
                   "order": wl.p, "precision": args.precision + ("-pop/f64-moments" if args.precision == "fp32" else ""),
                   "path": args.path, "path_resolved": s_path, "dt": wl.dt,
                   "nu": wl.nu, "seed": wl.meta.get("seed"), "unstable_flag": unstable},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(wname, args.precision, s_path),
                     "bytes_per_node_update": bpn,
                     "kernel": "stream+collide (one launch per step)",
                     "avg_kernel_ms": ms / args.steps},
    }
    if not args.no_fp64 and args.precision != "fp64":
        s64, ms64, _ = timed(wl, "fp64", args.path, args.steps, args.warmup)
        m32, m64 = s.moments(), s64.moments()

        def l2_rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out["fp64"] = {"value": s64.n * args.steps / (ms64 * 1e-3), "ms_per_step": ms64 / args.steps,
                       "bytes_per_node_update": bytes_per_node_update(wl, "fp64", s64.resolved_path()),
                       "traffic": profiled_traffic(wname, "fp64", s64.resolved_path()),
                       "fp32_vs_fp64_after_steps": {
                           "steps": args.warmup + args.steps,
                           "rho_max_rel": float(np.abs(m32[0] - m64[0]).max() / np.abs(m64[0]).max()),
                           "u_max_abs": float(max(np.abs(m32[1] - m64[1]).max(),
                                                  np.abs(m32[2] - m64[2]).max())),
                           "theta_max_rel": float(np.abs(m32[3] - m64[3]).max() / np.abs(m64[3]).max()),
                           "rho_l2_rel": l2_rel(m32[0], m64[0]),
                           "u_l2_rel": float(np.sqrt(((m32[1] - m64[1]) ** 2 + (m32[2] - m64[2]) ** 2).sum()
                                                     / (m64[1] ** 2 + m64[2] ** 2).sum())),
                           "theta_l2_rel": l2_rel(m32[3], m64[3]),
                           # zero-gradient boundaries: mass is not conserved, so these are
                           # changes over the run, and the FP32 - FP64 difference of the mass
                           "mass_rel_change_fp32": s.mass() / s.mass0 - 1.0,
                           "mass_rel_change_fp64": s64.mass() / s64.mass0 - 1.0,
                           "mass_fp32_vs_fp64_rel": s.mass() / s64.mass() - 1.0}}
        s64_moments = (m64, s64.mass() / s64.mass0 - 1.0)
        s64.close()
    else:
        s64_moments = None
    # initialisation, moments and mass on the same grid (this re-initialises s)
    out["aux_kernels"] = aux_kernels(s)
    if not args.no_mfma and args.precision == "fp32" and args.workload == "riemann":
        # the same step with the x-pass of the interpolation on the matrix cores
        sm, msm, _ = timed(wl, "fp32", "mfma", args.steps, args.warmup)
        v = sm.n * args.steps / (msm * 1e-3)
        out["mfma_x_pass"] = {"path": "mfma", "value": v, "unit": "node-updates/s",
                              "ms_per_step": msm / args.steps,
                              "achieved_gbs": v * bpn / 1e9, "frac": v * bpn / 1e9 / HBM_PEAK_GBS,
                              "mfma_tflops": v * mfma_flops_per_node_update(wl) / 1e12}
        sm.close()
    if not args.no_mfma and args.precision == "fp32" and args.workload == "riemann":
        out["bf16_experiment"] = bf16_experiment(wl, args.steps, args.warmup, s64_moments)
    if not args.no_mfma and args.workload == "riemann" and args.path == "auto":
        # the other LDS kernel family on the same workload (AUTO picks by measured speed)
        other = "tiled" if s_path == "rows" else "rows"
        so, mso, _ = timed(wl, args.precision, other, args.steps, args.warmup)
        v = so.n * args.steps / (mso * 1e-3)
        tro = profiled_traffic(wname, args.precision, other)
        out[f"{other}_path"] = {"path": other, "value": v, "unit": "node-updates/s",
                                "ms_per_step": mso / args.steps, "achieved_gbs": v * bpn / 1e9,
                                "frac": v * bpn / 1e9 / HBM_PEAK_GBS, "traffic": tro,
                                "traffic_over_algorithmic": tro / (so.n * bpn) if tro else None}
        so.close()
    if not args.no_svi and args.workload == "riemann":
        out["shock_vortex"] = shock_vortex_entry(args.precision)
        out["curvilinear"] = curvilinear_entry(args.precision)
        out["d3q125"] = d3q125_entry()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_cost()
        rec = adjoint_cost(every=0)
        out["adjoint"]["recorded_moments"] = {
            "note": "every step's moments kept in the forward (24 B per node and step), no replay",
            "forward_ms": rec["forward_ms"], "backward_ms": rec["backward_ms"], "ratio": rec["ratio"]}
    if not args.no_cpu_baseline:
        # same initial state, one GPU step, compared with the oracle at the sample
        s1 = Solver.from_workload(wl, precision=args.precision, path=args.path)
        s1.init_from_workload()
        s1.step(1)
        G1 = s1.populations().astype(np.float64)
        s1.close()
        cb, err = cpu_baseline(args.workload, G1)
        out["cpu_baseline"] = cb
        out["accuracy"] = {"one_step_max_rel_err_vs_fp64_oracle": err,
                           "sample_nodes": 250000}
    s.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
