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
  fcc128   the same sphere recipe on the FCC lattice (7 amplitudes: <111> and <200> shells, two-shell
           relaxed amplitudes), side 60 cubic constants, 20 steps

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tri1024|batch64|bcc128]
                    [--precision mixed|fp64] [--no-compare] [--no-variants] [--probe KERNEL] [--no-cpu-baseline]

Prints one JSON line; value = (sum over instances of J * N) * K / seconds of the K timed steps.  The
other precision runs the same steps afterwards (unless --no-compare) for the eta and energy differences.
With the default workload the line also carries `variants.batch64` and `variants.bcc128`: the same
K steps (after the same W warm-up steps) of the other two workloads, each with its own throughput,
roofline and mixed-vs-FP64 differences (--no-variants skips them).

Roofline: during the W warm-up steps the timing probe times every launch of every kernel family (HIP
events on the launch stream): `kernels` lists every family with a byte model (algorithmic bytes per
launch / average duration of its working launches) and its share of the kernel time.  The family with
the largest share is then sampled alone (every 7th launch) inside the timed region: `roofline`.
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
CSRC = os.path.join(ROOT, "paper_1902_09761_amd", "csrc")
KERNEL_SOURCES = ["apfc_internal.h", "kernels_common.h", "kernels.hip", "kernels_apply.hip", "kernels_cheb2d.hip",
                  "kernels_mg.hip", "kernels_mass.hip"]
PROFILES = os.path.join(ROOT, "profiles")
# kernel families with a byte model, as the library's probe names them, and the kernels they cover
FAMILIES = {"cheb": "k_cheb2d (3D: k_cb_*)", "apply": "k_apply_dot2d/3d", "proj_final": "k_proj_final",
            "residual": "k_residual2d/3d", "extrapolate": "k_extrapolate", "rhs": "k_rhs_nonlinear",
            "pcg_spmv": "k_cg_spmv", "pcg_update": "k_cg_update", "mass": "k_mass_sep"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's run length, 100 / 50 / 20)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tri1024", choices=["tri1024", "batch64", "bcc128", "fcc128"])
    ap.add_argument("--n", type=int, default=None, help="override the mesh side (tri1024 / bcc128)")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the run in the other precision (FP64 vs mixed: eta and energy differences)")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the batch64 and bcc128 runs that the default workload's line carries")
    ap.add_argument("--inner", default="cheb", choices=["pcg", "cheb", "mg"])
    ap.add_argument("--mass", default="sep", choices=["iter", "sep"],
                    help="step 1 of the preconditioner: inner iterations (iter) or the separable mass inverse "
                         "with --mass-iters taps per side (sep)")
    ap.add_argument("--restart", type=int, default=4)
    ap.add_argument("--x0", type=int, default=3, choices=[0, 1, 2, 3],
                    help="FGMRES initial guess: state of the last step (0) or its linear (1) / quadratic (2) / cubic (3) "
                         "extrapolation in time")
    ap.add_argument("--dt", type=float, default=None, help="time step (default: the workload's, 1.0)")
    ap.add_argument("--mass-iters", type=int, default=None)
    ap.add_argument("--diff-iters", type=int, default=None)
    ap.add_argument("--probe", default="all",
                    help="kernel family timed with HIP events for the roofline ('all': every family; 'none': off)")
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
    ap.add_argument("--study", default=None, choices=["dt"],
                    help="dt: the time-step sensitivity study on the chosen workload (one JSON line per time step "
                         "and inner-solver arm, then a markdown table); --steps and --warmup apply to every run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy 256 MiB device-to-device (reference for HBM counters)")
    return ap.parse_args()


def default_inner_iters(args):
    """(mass, diffusion) inner iterations: Chebyshev 5/3, multigrid 5 mass iterations and 2 smoothing
    iterations per side of each V-cycle, the paper's PCG 3/5; with the separable mass inverse the mass
    count is its taps per side (3)."""
    dm, dd = {"cheb": (5, 3), "mg": (5, 2)}.get(args.inner, (3, 5))
    if args.mass == "sep":
        dm = 3
    return args.mass_iters or dm, args.diff_iters or dd


_WORKLOADS = {}


def make_workload(args, workload):
    """Returns (lattice, list of inputs.Workload, dim); generated once per (workload, n) in a process."""
    key = (workload, args.n)
    if key not in _WORKLOADS:
        _WORKLOADS[key] = _make_workload(args, workload)
    return _WORKLOADS[key]


def _make_workload(args, workload):
    import numpy as np
    from paper_1902_09761_amd import apfc, inputs
    kind = {"bcc128": apfc.APFC_BCC3D, "fcc128": apfc.APFC_FCC3D}.get(workload, apfc.APFC_TRI2D)
    lat = apfc.apfc_lattice_default(kind)
    dim = 2 if kind == apfc.APFC_TRI2D else 3
    kk = np.array(apfc.lattice_k(lat, dim))

    def phi_of(dB):
        # one relaxed amplitude per amplitude (FCC: the <111> and <200> shells differ)
        return apfc.apfc_equilibrium_amplitudes(lat, apfc.apfc_params_default(a1=0.5 * dB))
    if workload == "tri1024":
        wls = [inputs.voronoi_2d(kk, phi_of, n=args.n or 1024, seed=1)]
    elif workload == "batch64":
        wls = inputs.batch_2d(kk, phi_of, count=64, seed=1)
    elif workload == "fcc128":
        wls = [inputs.sphere_3d(kk, phi_of, n=args.n or 128, seed=1, spacing=inputs.FCC_SPACING, name="fcc")]
    else:
        wls = [inputs.sphere_3d(kk, phi_of, n=args.n or 128, seed=1)]
    return lat, wls, dim


def run_gpu(args, precision, probe=None, workload=None, graphs=None):
    import torch
    from paper_1902_09761_amd import apfc, inputs
    workload = workload or args.workload
    lat, wls, dim = make_workload(args, workload)
    prec = apfc.APFC_MIXED if precision == "mixed" else apfc.APFC_FP64
    inner = {"cheb": apfc.APFC_INNER_CHEB, "mg": apfc.APFC_INNER_MG}.get(args.inner, apfc.APFC_INNER_PCG)
    mi, di = default_inner_iters(args)
    mk = apfc.APFC_MASS_SEPARABLE if args.mass == "sep" else apfc.APFC_MASS_ITER
    ps = [apfc.apfc_params_default(a1=0.5 * w.dB, rtol=1e-8, precision=prec, inner_kind=inner,
                                   restart=args.restart, mass_iters=mi, diff_iters=di, x0_order=args.x0,
                                   mass_kind=mk)
          for w in wls]
    ms = [apfc.make_mesh(dim, w.mesh.n, w.mesh.length) for w in wls]
    s = apfc.Solver(ms, lat, ps)
    graphs = args.graphs if graphs is None else graphs
    s.set_graphs(graphs)
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
    fam_probe = {}
    if args.warmup > 0:
        if probe == "all":
            # the warm-up steps sample every launch of every family: the per-family table and the family
            # with the largest share of the kernel time, which the timed region then samples alone
            s.probe_enable("all", 1)
        s.run(ets, zts, dt, args.warmup)
        if probe == "all":
            for f in FAMILIES:
                n, ms_, bpl, issued = s.probe_read_kernel(f)
                if n > 0:
                    fam_probe[f] = {"launches": n, "ms": ms_, "bytes_per_launch": bpl, "issued": issued}
            s.probe_read()
            s.probe_enable(None)
    if probe == "all":
        ranked = rooflines({"probe": fam_probe})
        probe = ranked[0]["family"] if ranked else "cheb"
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
           "relres": info["max_relres"], "instances": len(wls), "mesh": wls[0].name, "graphs": bool(graphs),
           "workload": workload}
    if probe:
        out["probe"] = {}
        n, ms_, bpl, issued = s.probe_read_kernel(probe)
        if n > 0:
            out["probe"][probe] = {"launches": n, "ms": ms_, "bytes_per_launch": bpl, "issued": issued}
        s.probe_read()
        s.probe_enable(None)
    out["warmup_probe"] = fam_probe
    out["energy"] = s.energy(ets)
    out["eta_host"] = [e.cpu().numpy() for e in ets]
    return out


def kernel_sources_sha256():
    """sha256 over the kernel sources (in the order of KERNEL_SOURCES): a counter summary is valid only
    for the kernels it was taken on."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def traffic_from_profile(family, workload, tiles):
    """HBM bytes per working launch of one kernel family from the committed counter summary
    profiles/<family>_<workload>_hbm_counters.md (one `traffic_bytes_per_launch[ROWS,REGION]` line per tiling
    measured), if it was taken with the current kernel source and the tiling the run used (null otherwise)."""
    path = os.path.join(PROFILES, f"{family}_{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    m2 = re.search(r"kernel_sources_sha256:\s*([0-9a-f]+)", text)
    rel = os.path.relpath(path, ROOT)
    if not m2 or m2.group(1) != kernel_sources_sha256():
        return None, rel
    for m in re.finditer(r"traffic_bytes_per_launch\[([0-9]+),([0-9]+)\]:\s*([0-9.]+)", text):
        if (int(m.group(1)), int(m.group(2))) == tuple(tiles):
            return float(m.group(3)), rel
    return None, rel


def rooflines(res):
    """Per-family roofline entries from the probe's samples, and the family with the largest share of the
    sampled kernel time (the dominant kernel)."""
    pr = res.get("probe") or {}
    fams = []
    for f, d in pr.items():
        if d["launches"] <= 0 or d["bytes_per_launch"] <= 0:
            continue
        avg_ms = d["ms"] / d["launches"]
        ach = d["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        fams.append({"family": f, "kernel": FAMILIES.get(f, f), "bytes_per_launch": d["bytes_per_launch"],
                     "avg_launch_us": 1e3 * avg_ms, "achieved": ach, "frac": ach / HBM_PEAK_GBS,
                     "sampled_launches": d["launches"], "issued": d["issued"],
                     # sampled time scaled by the sampling rate: the family's share of the kernel time
                     "est_ms": d["ms"] * d["issued"] / max(1, d["launches"])})
    fams.sort(key=lambda e: -e["est_ms"])
    tot = sum(e["est_ms"] for e in fams)
    for e in fams:
        e["time_share"] = e["est_ms"] / tot if tot > 0 else 0.0
    return fams


def roofline_entry(fam, workload, tiles, every):
    traffic, src = traffic_from_profile(fam["family"], workload, tiles)
    return {"bound": "hbm", "kernel": fam["kernel"], "family": fam["family"], "achieved": fam["achieved"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fam["frac"], "traffic": traffic, "traffic_source": src,
            "avg_launch_us": fam["avg_launch_us"], "launches": fam["sampled_launches"], "sampled_every": every,
            "bytes_per_launch": fam["bytes_per_launch"], "time_share": fam["time_share"]}


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


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
    h = host_info()
    return {"value": len(k) * wl.mesh.N / sec, "unit": "amplitude-DOF-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}; SuperLU factor + solve per amplitude, single-threaded; {sec:.1f} s",
            "host_cpu": h["cpu_model"], "host_nproc": h["nproc"]}


def measure(args, workload, precision, probe, compare, graphs=None):
    """One workload: the timed run, its rooflines and (compare) the other precision's run of the same
    steps.  Returns the fields of a bench line (or of a variant)."""
    import numpy as np
    res = run_gpu(args, precision, probe=probe, workload=workload, graphs=graphs)
    K = args.steps
    out = {"value": res["dofs"] * K / res["sec"], "ms_per_step": 1e3 * res["sec"] / K,
           "fgmres_iters_per_step": float(np.mean(res["iters"])), "final_relres": res["relres"],
           "config": {"workload": workload, "instances": res["instances"], "first_instance": res["mesh"],
                      "amplitude_dofs": res["dofs"], "J": res["J"], "dt": res["dt"], "rtol": 1e-8,
                      "precision": precision, "inner": args.inner, "restart": args.restart,
                      "tile_rows": res["tile_rows"][0], "precond_region": res["tile_rows"][1],
                      "mass": args.mass, "mass_iters": default_inner_iters(args)[0],
                      "diff_iters": default_inner_iters(args)[1],
                      "x0_order": args.x0,
                      "graphs": res["graphs"], "entry": "apfc_step" if args.per_step else "apfc_run"}}
    timed = rooflines(res)
    if timed:
        out["roofline"] = roofline_entry(timed[0], workload, res["tile_rows"], args.probe_every)
    listed = rooflines({"probe": res["warmup_probe"]})
    if timed:
        share = [e["time_share"] for e in listed if e["family"] == timed[0]["family"]]
        out["roofline"]["time_share"] = share[0] if share else None
    if listed:
        # every family with a byte model, from the warm-up steps (every launch timed)
        out["kernels"] = [{k: e[k] for k in ("family", "kernel", "bytes_per_launch", "avg_launch_us", "achieved",
                                             "frac", "time_share", "sampled_launches")} for e in listed]
    if compare:
        other = "fp64" if precision == "mixed" else "mixed"
        r2 = run_gpu(args, other, workload=workload, graphs=graphs)
        a, b = (res, r2) if precision == "fp64" else (r2, res)
        diffs = [float(np.linalg.norm(y - x) / np.linalg.norm(x)) for x, y in zip(a["eta_host"], b["eta_host"])]
        ediff = [abs(y - x) / abs(x) for x, y in zip(a["energy"], b["energy"])]
        out["other_precision"] = {other: {"value": res["dofs"] * K / r2["sec"], "ms_per_step": 1e3 * r2["sec"] / K,
                                          "fgmres_iters_per_step": float(np.mean(r2["iters"]))},
                                  "mixed_vs_fp64_eta_rel_l2": max(diffs),
                                  "mixed_vs_fp64_energy_rel": max(ediff)}
    return out


STUDY_DT = [0.1, 0.3, 1.0, 3.0, 10.0, 30.0, 100.0]
# (label, inner solver, mass step, mass iterations or taps, diffusion iterations or smoothing iterations,
#  initial-guess order, time steps)
STUDY_ARMS = [("PCG 3/5 (paper), x0 0", "pcg", "iter", 3, 5, 0, STUDY_DT),
              ("Chebyshev 5/3, x0 0", "cheb", "iter", 5, 3, 0, STUDY_DT),
              ("separable 3 + Chebyshev 3, x0 0", "cheb", "sep", 3, 3, 0, STUDY_DT),
              ("separable 3 + Chebyshev 3, x0 3", "cheb", "sep", 3, 3, 3, STUDY_DT),
              ("separable 3 + Chebyshev 6, x0 0", "cheb", "sep", 3, 6, 0, STUDY_DT),
              ("separable 3 + multigrid nu=1, x0 0", "mg", "sep", 3, 1, 0, STUDY_DT),
              ("separable 3 + multigrid nu=2, x0 0", "mg", "sep", 3, 2, 0, STUDY_DT),
              ("PCG 20/20 (inner solves ~exact), x0 0", "pcg", "iter", 20, 20, 0, [1.0, 10.0, 100.0])]


def dt_study(args):
    """FGMRES iterations per step (slowest system) and wall time per step against dt for each inner-solver
    arm: the analogue of the paper's Fig. 4(a).  Prints one JSON line per run, then a markdown table."""
    import numpy as np
    rows = {}
    for label, inner, mass, mi, di, x0, dts in STUDY_ARMS:
        for dt in dts:
            args.inner, args.mass, args.mass_iters, args.diff_iters, args.x0, args.dt = inner, mass, mi, di, x0, dt
            try:
                res = run_gpu(args, args.precision, probe=None)
            except Exception as e:      # e.g. FGMRES reached max_iters on this arm
                print(json.dumps({"arm": label, "dt": dt, "error": str(e)}), flush=True)
                continue
            r = {"arm": label, "dt": dt, "ms_per_step": 1e3 * res["sec"] / args.steps,
                 "fgmres_iters_per_step": float(np.mean(res["iters"])), "final_relres": res["relres"],
                 "workload": res["workload"], "steps": args.steps, "warmup": args.warmup,
                 "tiles": res["tile_rows"]}
            rows[(label, dt)] = r
            print(json.dumps(r), flush=True)
    print("| dt | " + " | ".join(a[0] for a in STUDY_ARMS) + " |")
    print("|---" * (len(STUDY_ARMS) + 1) + "|")
    for dt in STUDY_DT:
        cells = []
        for a in STUDY_ARMS:
            r = rows.get((a[0], dt))
            cells.append("—" if r is None else f"{r['fgmres_iters_per_step']:.1f} its, {r['ms_per_step']:.2f} ms")
        print(f"| {dt:g} | " + " | ".join(cells) + " |", flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.study == "dt":
        if args.steps is None:
            args.steps = 10
        dt_study(args)
        return
    if args.steps is None:
        args.steps = {"tri1024": 100, "batch64": 50, "bcc128": 20, "fcc128": 20}[args.workload]
    probe = None if args.probe in ("", "none") else args.probe
    K = args.steps
    m = measure(args, args.workload, args.precision, probe, args.compare)
    line = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "amplitude-DOF-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": m["config"],
        "fgmres_iters_per_step": m["fgmres_iters_per_step"],
        "final_relres": m["final_relres"],
    }
    for key in ("roofline", "kernels"):
        if key in m:
            line[key] = m[key]
    variants = {}
    if "other_precision" in m:
        variants.update(m["other_precision"])
    if args.variants and args.workload == "tri1024" and args.n is None:
        for wl in ("batch64", "bcc128", "fcc128"):
            v = measure(args, wl, args.precision, probe, args.compare)
            v.pop("kernels", None)
            variants[wl] = v
    if variants:
        line["variants"] = variants
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
