"""Throughput of the APFC time step on one MI355X.

A step is one time step of Algorithm 1 with K = 1 (nodal nonlinearity, right-hand sides, then
restarted FGMRES with the block preconditioner on every amplitude to ||b - A x|| <= 1e-8 ||b||); the
K timed steps run in one apfc_run call (--per-step: one apfc_step call each).
Workloads (seeded, synthetic, resident in HBM before the timed region starts):

  tri1024  (default) 1024^2 triangular-lattice polycrystal, 16 periodic Voronoi grains within +-10
           degrees, side 400 lattice spacings, 3 amplitudes, dt = 1, 100 steps
  batch64  64 independent triangular instances of seeded size n^2, n in {128,...,512}, one rotated grain
           each, Delta B ~ U[0.01, 0.05], all in one batched context, 50 steps
  bcc128   128^3 bcc lattice (6 amplitudes), spherical grain rotated 5 degrees about [001], 20 steps

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tri1024|batch64|bcc128]
                    [--precision mixed|fp64] [--no-compare] [--probe KERNEL] [--no-cpu-baseline]

Prints one JSON line; value = (sum over instances of J * N) * K / seconds of the K timed steps.  The
other precision runs the same steps afterwards (unless --no-compare) for the eta and energy differences.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude DOF-steps/s at 1e-8 rel. residual + % HBM peak; plain vs mixed/batch"
HBM_PEAK_GBS = 8000.0
KERNELS_SRC = os.path.join(ROOT, "paper_1902_09761_amd", "csrc", "kernels.hip")
TRAFFIC_MD = os.path.join(ROOT, "profiles", "apply_dot_tri1024_mixed_hbm_counters.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's run length, 100 / 50 / 20)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tri1024", choices=["tri1024", "batch64", "bcc128"])
    ap.add_argument("--n", type=int, default=None, help="override the mesh side (tri1024 / bcc128)")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the run in the other precision (FP64 vs mixed: eta and energy differences)")
    ap.add_argument("--inner", default="cheb", choices=["pcg", "cheb"])
    ap.add_argument("--restart", type=int, default=4)
    ap.add_argument("--x0", type=int, default=3, choices=[0, 1, 2, 3],
                    help="FGMRES initial guess: state of the last step (0) or its linear (1) / quadratic (2) / cubic (3) "
                         "extrapolation in time")
    ap.add_argument("--dt", type=float, default=None, help="time step (default: the workload's, 1.0)")
    ap.add_argument("--mass-iters", type=int, default=None)
    ap.add_argument("--diff-iters", type=int, default=None)
    ap.add_argument("--probe", default="apply", help="kernel timed with HIP events for the roofline ('none': off)")
    ap.add_argument("--probe-every", type=int, default=7,
                    help="time every n-th launch of the probed kernel (an event pair idles the stream briefly; "
                         "keep n coprime with the restart length so that every Arnoldi index is sampled)")
    ap.add_argument("--graphs", action="store_true", help="replay restart cycles as hipGraphs")
    ap.add_argument("--per-step", action="store_true",
                    help="one apfc_step call per step instead of one apfc_run call for the K steps")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tiles", default=None,
                    help="ROWS[,REGION]: fixed tile rows (and fused-preconditioner region) instead of the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy 256 MiB device-to-device (reference for HBM counters)")
    return ap.parse_args()


def make_workload(args):
    """Returns (lattice, list of inputs.Workload, dim)."""
    import numpy as np
    from paper_1902_09761_amd import apfc, inputs
    kind = apfc.APFC_BCC3D if args.workload == "bcc128" else apfc.APFC_TRI2D
    lat = apfc.apfc_lattice_default(kind)
    dim = 3 if kind == apfc.APFC_BCC3D else 2
    kk = np.array(apfc.lattice_k(lat, dim))

    def phi_of(dB):
        return apfc.apfc_uniform_amplitude(lat, apfc.apfc_params_default(a1=0.5 * dB))
    if args.workload == "tri1024":
        wls = [inputs.voronoi_2d(kk, phi_of, n=args.n or 1024, seed=1)]
    elif args.workload == "batch64":
        wls = inputs.batch_2d(kk, phi_of, count=64, seed=1)
    else:
        wls = [inputs.sphere_3d(kk, phi_of, n=args.n or 128, seed=1)]
    return lat, wls, dim


def run_gpu(args, precision, probe=None):
    import torch
    from paper_1902_09761_amd import apfc, inputs
    lat, wls, dim = make_workload(args)
    prec = apfc.APFC_MIXED if precision == "mixed" else apfc.APFC_FP64
    inner = apfc.APFC_INNER_CHEB if args.inner == "cheb" else apfc.APFC_INNER_PCG
    mi = args.mass_iters or (5 if args.inner == "cheb" else 3)
    di = args.diff_iters or (3 if args.inner == "cheb" else 5)
    ps = [apfc.apfc_params_default(a1=0.5 * w.dB, rtol=1e-8, precision=prec, inner_kind=inner,
                                   restart=args.restart, mass_iters=mi, diff_iters=di, x0_order=args.x0)
          for w in wls]
    ms = [apfc.make_mesh(dim, w.mesh.n, w.mesh.length) for w in wls]
    s = apfc.Solver(ms, lat, ps)
    s.set_graphs(args.graphs)
    if args.tiles:
        tr = [int(v) for v in args.tiles.split(",")]
        s.set_tiles(tr[0], tr[1] if len(tr) > 1 else 0)
    elif not args.no_autotune:
        s.autotune()
    ty = s.get_tiles()
    ets = [torch.tensor(inputs.to_planar(w.eta0), dtype=torch.float64, device="cuda") for w in wls]
    zts = [torch.zeros_like(e) for e in ets]
    s.init_zeta(ets, zts)
    dt = args.dt if args.dt is not None else wls[0].dt
    if args.warmup > 0:
        s.run(ets, zts, dt, args.warmup)
    if probe:
        s.probe_enable(probe, args.probe_every)
    iters, total = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.per_step:
        for _ in range(args.steps):
            info = s.step(ets, zts, dt)
            iters.append(info["max_iters"])
            total.append(info["total_iters"])
    else:
        info = s.run(ets, zts, dt, args.steps)
        iters = info["step_max_iters"]
        total = [info["total_iters"]]
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    J = lat.J
    dofs = sum(J * w.mesh.N for w in wls)
    out = {"sec": sec, "iters": iters, "total_iters": total, "tile_rows": ty, "dofs": dofs, "J": J, "dt": dt,
           "relres": info["max_relres"], "instances": len(wls), "mesh": wls[0].name}
    if probe:
        n, ms_, bpl = s.probe_read()
        out["probe"] = {"kernel": probe, "launches": n, "ms": ms_, "bytes_per_launch": bpl,
                        "every": args.probe_every}
        s.probe_enable(None)
    out["energy"] = s.energy(ets)
    out["eta_host"] = [e.cpu().numpy() for e in ets]
    return out


def traffic_from_profile(tile_rows):
    """HBM bytes per k_apply_dot launch from the committed counter summary, if it was taken with the
    current kernel source and the same tile rows (null otherwise)."""
    if not os.path.exists(TRAFFIC_MD):
        return None, None
    text = open(TRAFFIC_MD).read()
    m1 = re.search(r"traffic_bytes_per_launch:\s*([0-9.]+)", text)
    m2 = re.search(r"kernels_hip_sha256:\s*([0-9a-f]+)", text)
    m3 = re.search(r"tile_rows:\s*([0-9]+)", text)
    sha = hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest()
    if not (m1 and m2 and m3) or m2.group(1) != sha or int(m3.group(1)) != tile_rows:
        return None, os.path.relpath(TRAFFIC_MD, ROOT)
    return float(m1.group(1)), os.path.relpath(TRAFFIC_MD, ROOT)


def cpu_baseline(args):
    """The oracle (SuperLU factor + solve per amplitude, single-threaded) on one step of the same
    workload recipe at a reduced size with the same h."""
    from oracle.apfc_oracle import BulkEnergy, Grid, Oracle, Params, bcc_k, tri_k, uniform_amplitude
    from paper_1902_09761_amd import inputs
    if args.workload == "bcc128":
        k, n = bcc_k(), 16
        wl = inputs.sphere_3d(k, lambda dB: uniform_amplitude(BulkEnergy(k, Params.from_dB(dB))), n=n, seed=1)
        what = f"1 step of the bcc sphere recipe at {n}^3 nodes (same h, 6 amplitudes)"
    else:
        k, n = tri_k(), 192
        wl = inputs.voronoi_2d(k, lambda dB: uniform_amplitude(BulkEnergy(k, Params.from_dB(dB))), n=n, seed=1)
        what = f"1 step of the Voronoi recipe at {n}^2 nodes (same h, 3 amplitudes)"
    o = Oracle(Grid(wl.mesh.dim, wl.mesh.n[: wl.mesh.dim], wl.mesh.length[: wl.mesh.dim]), k, Params.from_dB(wl.dB))
    t0 = time.perf_counter()
    o.step(wl.eta0, args.dt if args.dt is not None else wl.dt)
    sec = time.perf_counter() - t0
    return {"value": len(k) * wl.mesh.N / sec, "unit": "amplitude-DOF-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}; SuperLU factor + solve per amplitude, single-threaded; {sec:.1f} s"}


def main():
    args = parse()
    if args.steps is None:
        args.steps = {"tri1024": 100, "batch64": 50, "bcc128": 20}[args.workload]
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    probe = None if args.probe in ("", "none") else args.probe
    res = run_gpu(args, args.precision, probe=probe)
    K = args.steps
    value = res["dofs"] * K / res["sec"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitude-DOF-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * res["sec"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "instances": res["instances"], "first_instance": res["mesh"],
                   "amplitude_dofs": res["dofs"], "J": res["J"], "dt": res["dt"], "rtol": 1e-8,
                   "precision": args.precision, "inner": args.inner, "restart": args.restart,
                   "tile_rows": res["tile_rows"][0], "precond_region": res["tile_rows"][1],
                   "mass_iters": args.mass_iters or (5 if args.inner == "cheb" else 3),
                   "diff_iters": args.diff_iters or (3 if args.inner == "cheb" else 5), "x0_order": args.x0,
                   "graphs": bool(args.graphs), "entry": "apfc_step" if args.per_step else "apfc_run"},
        "fgmres_iters_per_step": float(np.mean(res["iters"])),
        "final_relres": res["relres"],
    }
    pr = res.get("probe")
    if pr and pr["launches"] > 0:
        avg_ms = pr["ms"] / pr["launches"]
        ach = pr["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        traffic, src = (traffic_from_profile(res["tile_rows"][0])
                        if (pr["kernel"] == "apply" and args.workload == "tri1024" and args.precision == "mixed")
                        else (None, None))
        line["roofline"] = {"bound": "hbm", "kernel": "k_apply_dot" if pr["kernel"] == "apply" else pr["kernel"],
                            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                            "traffic": traffic, "traffic_source": src, "avg_launch_us": 1e3 * avg_ms,
                            "launches": pr["launches"], "sampled_every": pr["every"],
                            "bytes_per_launch": pr["bytes_per_launch"]}
    if args.compare:
        other = "fp64" if args.precision == "mixed" else "mixed"
        r2 = run_gpu(args, other)
        a, b = (res, r2) if args.precision == "fp64" else (r2, res)
        diffs = [float(np.linalg.norm(y - x) / np.linalg.norm(x)) for x, y in zip(a["eta_host"], b["eta_host"])]
        ediff = [abs(y - x) / abs(x) for x, y in zip(a["energy"], b["energy"])]
        line["variants"] = {other: {"value": res["dofs"] * K / r2["sec"], "ms_per_step": 1e3 * r2["sec"] / K,
                                    "fgmres_iters_per_step": float(np.mean(r2["iters"]))},
                            "mixed_vs_fp64_eta_rel_l2": max(diffs),
                            "mixed_vs_fp64_energy_rel": max(ediff)}
    if args.calibrate_copy:
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
