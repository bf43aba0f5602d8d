"""Throughput of the APFC time step on one MI355X.

A step is one apfc_step (Algorithm 1 with K = 1: nodal nonlinearity, then restarted FGMRES with
the block preconditioner on every amplitude to rtol 1e-8) on the 1024^2 triangular-lattice
polycrystal (16 periodic Voronoi grains within +-10 degrees, side 400 lattice spacings, dt = 1).
Inputs are seeded and synthetic and live in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
                    [--probe KERNEL] [--no-cpu-baseline]

Prints one JSON line.  value = J * N * K / (seconds of the K timed steps).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitude DOF-steps/s at 1e-8 rel. residual + % HBM peak; plain vs mixed/batch"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--compare", action="store_true", help="also time the other precision")
    ap.add_argument("--inner", default="cheb", choices=["pcg", "cheb"])
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--mass-iters", type=int, default=None)
    ap.add_argument("--diff-iters", type=int, default=None)
    ap.add_argument("--probe", default="pcg_spmv", help="kernel timed with HIP events for the roofline")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=192, help="mesh side of the oracle sample")
    return ap.parse_args()


def make_workload(n):
    from paper_1902_09761_amd import apfc, inputs
    lat = apfc.apfc_lattice_default(apfc.APFC_TRI2D)
    k = apfc.lattice_k(lat, 2)
    import numpy as np
    kk = np.array(k)

    def phi_of(dB):
        return apfc.apfc_uniform_amplitude(lat, apfc.apfc_params_default(a1=0.5 * dB))
    return inputs.voronoi_2d(kk, phi_of, n=n, seed=1), lat


def run_gpu(args, precision, probe=None):
    import torch
    from paper_1902_09761_amd import apfc, inputs
    wl, lat = make_workload(args.n)
    prec = apfc.APFC_MIXED if precision == "mixed" else apfc.APFC_FP64
    inner = apfc.APFC_INNER_CHEB if args.inner == "cheb" else apfc.APFC_INNER_PCG
    mi = args.mass_iters or (4 if args.inner == "cheb" else 3)
    di = args.diff_iters or (4 if args.inner == "cheb" else 5)
    p = apfc.apfc_params_default(a1=0.5 * wl.dB, rtol=wl.rtol, precision=prec, inner_kind=inner,
                                 restart=args.restart, mass_iters=mi, diff_iters=di)
    m = apfc.make_mesh(2, wl.mesh.n, wl.mesh.length)
    s = apfc.Solver([m], lat, [p])
    if args.no_graphs:
        s.set_graphs(False)
    ty = None if args.no_autotune else s.autotune()
    et = torch.tensor(inputs.to_planar(wl.eta0), dtype=torch.float64, device="cuda")
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    for _ in range(args.warmup):
        s.step([et], [zt], wl.dt)
    if probe:
        s.probe_enable(probe)
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = s.step([et], [zt], wl.dt)
        iters.append(info["max_iters"])
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out = {"sec": sec, "iters": iters, "tile_rows": ty, "N": wl.mesh.N, "J": 3, "relres": info["max_relres"]}
    if probe:
        n, ms, bpl = s.probe_read()
        out["probe"] = {"kernel": probe, "launches": n, "ms": ms, "bytes_per_launch": bpl}
        s.probe_enable(None)
    E = s.energy([et])[0]
    out["energy"] = E
    out["eta_host"] = et.cpu().numpy()
    return out


def cpu_baseline(args):
    """The oracle (SuperLU direct solves, single-threaded) on one step of the same workload recipe
    at a reduced mesh side with the same h."""
    import numpy as np
    from oracle.apfc_oracle import BulkEnergy, Grid, Oracle, Params, tri_k, uniform_amplitude
    from paper_1902_09761_amd import inputs
    n = args.cpu_n
    wl = inputs.voronoi_2d(tri_k(), lambda dB: uniform_amplitude(BulkEnergy(tri_k(), Params.from_dB(dB))), n=n, seed=1)
    o = Oracle(Grid(2, (n, n), wl.mesh.length[:2]), tri_k(), Params.from_dB(wl.dB))
    t0 = time.perf_counter()
    o.step(wl.eta0, wl.dt)
    sec = time.perf_counter() - t0
    return {"value": 3 * n * n / sec, "unit": "amplitude-DOF-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of the Voronoi recipe at {n}^2 nodes (same h, 3 amplitudes; SuperLU "
                      f"factor+solve per amplitude, single-threaded), {sec:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    probe = None if args.probe in ("", "none") else args.probe
    res = run_gpu(args, args.precision, probe=probe)
    J, N, K = res["J"], res["N"], args.steps
    value = J * N * K / res["sec"]
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
        "config": {"workload": f"tri{args.n}_voronoi16", "mesh": f"{args.n}x{args.n} periodic Q1", "J": 3,
                   "dt": 1.0, "rtol": 1e-8, "precision": args.precision, "restart": args.restart,
                   "inner": args.inner, "tile_rows": res["tile_rows"],
                   "graphs": not args.no_graphs},
        "fgmres_iters_per_step": float(np.mean(res["iters"])),
        "final_relres": res["relres"],
    }
    pr = res.get("probe")
    if pr and pr["launches"] > 0:
        avg_ms = pr["ms"] / pr["launches"]
        ach = pr["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        line["roofline"] = {"bound": "hbm", "kernel": pr["kernel"], "achieved": ach, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                            "avg_launch_us": 1e3 * avg_ms, "launches": pr["launches"],
                            "bytes_per_launch": pr["bytes_per_launch"]}
    if args.compare:
        other = "fp64" if args.precision == "mixed" else "mixed"
        r2 = run_gpu(args, other)
        v2 = J * N * K / r2["sec"]
        a, b = (res, r2) if args.precision == "fp64" else (r2, res)
        diff = float(np.linalg.norm(b["eta_host"] - a["eta_host"]) / np.linalg.norm(a["eta_host"]))
        line["variants"] = {other: {"value": v2, "ms_per_step": 1e3 * r2["sec"] / K,
                                    "fgmres_iters_per_step": float(np.mean(r2["iters"]))},
                            "mixed_vs_fp64_eta_rel_l2": diff,
                            "mixed_vs_fp64_energy_rel": abs(b["energy"] - a["energy"]) / abs(a["energy"])}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
