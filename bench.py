"""Throughput benchmark of the fluctuating D3Q19 lattice Boltzmann step on one
MI355X.

Workload: a 512^3 periodic box, fp32 deviation storage updated in place (AA
pattern, one buffer of 10.2 GB), rho0 = 1, kT = 1e-4, gamma_shear = 0.8,
gamma_bulk = 0.5, kinetic rates 0, thermal (random seeded rest) start with
Philox seed 1234.  One step = the whole fused collide-and-stream update of
every site.  The same box is also timed with fp16 and bf16 storage, and the
96-replica ensemble in one launch per step.

Prints one JSON line.  `value` is MLUPS (million lattice-site updates per
second) of the fp32 run with the state resident in HBM; `roofline` compares
the step kernel's algorithmic bytes (19 populations read and written, 2 * 19
* 4 bytes per site) per launch, divided by the mean launch duration measured
with HIP events on the kernel's stream, with the 8 TB/s HBM peak; the mode
variances of the final state are checked against mu rho w_k (the stationary
law), and `cpu_baseline` times the FP64 CPU oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
W36 = [36, 12, 12, 12, 24, 48, 16, 4, 4, 4, 24, 24, 24, 8, 8, 8, 72, 48, 16]  # 36 w_k, Table II
KERNEL_SOURCES = ["paper_0707_1581_amd/csrc/lbf_kernels.h", "paper_0707_1581_amd/csrc/lbf_math.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_aa_step_512.json")


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(storage):
    """HBM bytes per step launch measured by rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy kernel), if taken on the current kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(storage)


def time_steps(step, steps, warmup, sync_stream):
    import torch
    step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sync_stream)
    step(steps)
    e1.record(sync_stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def mode_variance_dev(lat, rho0, kT):
    """max_k |var(m_k - m_k^eq) / (mu rho_mean w_k) - 1| of the current state
    (conserved modes about their lattice mean)."""
    import torch
    m = lat.modes()
    mu = 3.0 * kT
    rho = rho0 + m[0].double()
    rbar = float(rho.mean())
    j = m[1:4].double()
    worst = 0.0
    for k in range(19):
        x = m[k].double()
        if 4 <= k <= 9:
            jx, jy, jz = j[0], j[1], j[2]
            eq = {4: jx * jx + jy * jy + jz * jz, 5: 2 * jx * jx - jy * jy - jz * jz,
                  6: jy * jy - jz * jz, 7: jx * jy, 8: jy * jz, 9: jz * jx}[k] / rho
            x = x - eq
        var = float(((x - x.mean()) ** 2).mean()) if k < 4 else float((x ** 2).mean() - x.mean() ** 2)
        worst = max(worst, abs(var / (mu * rbar * W36[k] / 36.0) - 1.0))
        del x
    del m, rho, j
    torch.cuda.empty_cache()
    return worst


def run_lattice(box, storage, steps, warmup, cfg, check=True):
    import torch
    import paper_0707_1581_amd as lbf
    lat = lbf.Lattice(box, box, box, storage=storage, init="thermal", **cfg)
    sites = box ** 3
    ms = time_steps(lat.step, steps, warmup, lat.stream)
    bpe = 4 if storage == "f32" else 2
    alg = 2 * 19 * bpe * sites  # algorithmic bytes per step launch
    out = dict(storage=storage, ms_per_step=ms, mlups=sites / ms / 1e3,
               achieved_gbs=alg / ms / 1e6, alg_bytes_per_launch=alg)
    if check:
        nb, sums = lat.check()
        out["bad_sites"] = nb
        out["mode_variance_max_dev"] = mode_variance_dev(lat, cfg["rho0"], cfg["kT"])
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def run_ensemble(storage, steps, warmup):
    import torch
    import paper_0707_1581_amd as lbf
    import workloads
    reps = workloads.ensemble_replicas()
    ens = lbf.Ensemble(reps, storage=storage, init="thermal")
    ms = time_steps(ens.step, steps, warmup, ens.stream)
    sites = ens.sites()
    out = dict(storage=storage, replicas=len(reps), sites=sites, ms_per_step=ms,
               mlups=sites / ms / 1e3, schedule=ens.schedule())
    ens.close()
    del ens
    torch.cuda.empty_cache()
    return out


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle on the host cores: a 128^3 box from a thermal start,
    as many steps as fit in the budget (at least one)."""
    import oracle
    import workloads
    cfg = dict(workloads.MID, kT=1e-4, gamma_shear=0.8)
    p = oracle.params(**{k: cfg[k] for k in ("nx", "ny", "nz", "rho0", "kT", "gamma_bulk",
                                             "gamma_shear", "gamma_odd", "gamma_even", "seed")})
    n = oracle.init(p, oracle.INIT_THERMAL)
    sites = cfg["nx"] * cfg["ny"] * cfg["nz"]
    t0 = time.perf_counter()
    n = oracle.run(p, n, 0, 1)
    one = time.perf_counter() - t0
    k = max(1, int(budget_s / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    n = oracle.run(p, n, 1, k)
    dt = time.perf_counter() - t0
    return {"value": sites * k / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"128^3 box, thermal start, kT=1e-4, gamma_shear=0.8, {k} steps after 1 warm-up "
                      f"step, FP64 two-buffer push, {dt:.1f} s"}


def copy_calibration(gib=4):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the profiler."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 4 * n}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--box", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true", help="time only the fp32 box")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 4 GiB device copy (profiler counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "the update is a single-device kernel (see DESIGN.md for how it would shard)"}),
              flush=True)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    import paper_0707_1581_amd as lbf
    lbf.lib()

    import workloads
    cfg = {k: workloads.LARGE[k] for k in ("rho0", "kT", "gamma_bulk", "gamma_shear", "gamma_odd",
                                          "gamma_even", "seed")}
    main_run = run_lattice(args.box, "f32", args.steps, args.warmup, cfg)
    variants = {}
    if not args.no_variants:
        for st in ("f16", "bf16"):
            r = run_lattice(args.box, st, args.steps, args.warmup, cfg)
            r["roofline_frac"] = r["achieved_gbs"] / HBM_PEAK_GBS
            r["gain_over_f32"] = r["mlups"] / main_run["mlups"]
            variants[st] = r
        for st in ("f32", "f16"):
            variants[f"ensemble96_{st}"] = run_ensemble(st, max(20, args.steps), args.warmup)
    if args.copy_calibration:
        copy_calibration()

    traffic = stored_traffic("f32")
    roofline = {"bound": "hbm", "achieved": main_run["achieved_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": main_run["achieved_gbs"] / HBM_PEAK_GBS,
                "traffic": traffic,
                "kernel": "lbf::k_step<fp32> (even and odd AA launches; mean launch duration)",
                "alg_bytes_per_launch": main_run["alg_bytes_per_launch"]}
    line = {
        "metric": "MLUPS and % HBM roofline, FP32 vs 16-bit storage at 1% mode-variance error",
        "value": main_run["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 fluctuating LB, {args.box}^3 periodic box, fp32 AA in-place single "
                               f"buffer, rho0=1, kT=1e-4, gamma_shear=0.8, gamma_bulk=0.5, kinetic rates 0, "
                               f"thermal start, Philox seed 1234",
                   "sites": args.box ** 3, "storage": "f32",
                   "mode_variance_max_dev": main_run["mode_variance_max_dev"],
                   "bad_sites": main_run["bad_sites"]},
        "roofline": roofline,
        "variants": variants,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
