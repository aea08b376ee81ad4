"""Throughput of the thermal pseudopotential D3Q19 step on one MI355X.

Workload: the 512^3 boiling convection cell in FP32 (walls at z, periodic x, y;
mean density inside the coexistence region at the bottom-wall temperature),
the paper's resolution (L = 512, Table 1).  A step is one full lattice update
(every step of the hot path: moments, pseudopotential and thermal forces,
both BGK collisions with the counter-term, streaming and the walls) with the
populations resident in HBM.

Prints one JSON line: MLUPS, ms per step, the roofline of the step kernel
(algorithmic bytes = 38 reads + 38 writes of stored populations per node),
the FP16/BF16-deviation storage forms beside it, and the FP64 CPU oracle
timed on a bounded sample on the host.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + achieved HBM GB/s (% of peak), FP32 vs FP16-storage, 512^3 boiling"
PEAK_HBM_GBS = 8000.0
BYTES_PER_POP = {"fp64": 8, "fp32": 4, "fp16dev": 2, "bf16dev": 2}

TC = 0.05                              # critical temperature (sets G)
NU = 0.0165                            # kinematic viscosity, Table 1
TAU_NU = 0.5 + 3 * NU                  # 0.5495
TAU_KAPPA = 0.6417                     # Pr = 9 in the liquid at the mid temperature
RHO_BOIL = 1.93                        # liquid-rich mean density, boils at the bottom wall
GRAVITY = 3.2e-6


def workload_params(lbm, n, storage, kernel=0, tile_y=0, z_chunk=0, tile_x=0):
    return lbm.Params(
        n, n, n, storage=lbm.STORAGE[storage], kernel=kernel, tile_x=tile_x, tile_y=tile_y,
        z_chunk=z_chunk,
        tau_nu=TAU_NU, tau_kappa=TAU_KAPPA, G=-TC * math.e ** 2, T_d=0.95 * TC, T_u=0.85 * TC,
        gravity=GRAVITY, c_v=1.0, rho_kappa=0.5, rho_ref=RHO_BOIL, T_ref=0.9 * TC)


def time_steps(lat, steps, warmup):
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = lat.h.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def run_storage(lbm, n, storage, steps, warmup, rho0, kernel=0, tile_y=0, z_chunk=0, tile_x=0):
    import torch
    p = workload_params(lbm, n, storage, kernel, tile_y, z_chunk, tile_x)
    lat = lbm.Lattice(p, rho0)
    ms, wall = time_steps(lat, steps, warmup)
    tot = lat.moments()          # also checks the state is finite
    nodes = n ** 3
    bpn = 2 * 38 * BYTES_PER_POP[storage]
    res = {
        "mlups": nodes / (ms * 1e-3) / 1e6,
        "ms_per_step": ms,
        "achieved_gbs": bpn * nodes / (ms * 1e-3) / 1e9,
        "bytes_per_node": bpn,
        "mass_drift": None,
        "wall_s": wall,
    }
    del lat
    torch.cuda.empty_cache()
    return res, tot


def source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1111_0905_amd", "csrc", "*.hip")) +
                    glob.glob(os.path.join(ROOT, "paper_1111_0905_amd", "csrc", "*.hpp"))):
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(storage, n):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on this very kernel source and workload (else None)."""
    path = os.path.join(ROOT, "profiles", f"k_fused_{storage}_{n}cubed_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha256") != source_hash():
        return None
    return d["traffic_bytes_per_launch"]


def cpu_baseline(seconds=15.0):
    """FP64 oracle on the host, 64^3 sample of the same physics."""
    import torch
    import synth
    from oracle import lbm as olbm
    threads = os.cpu_count() or 1
    torch.set_num_threads(threads)
    n = 64
    p = olbm.Params(n, n, n, tau_nu=TAU_NU, tau_kappa=TAU_KAPPA, G=-TC * math.e ** 2,
                    T_d=0.95 * TC, T_u=0.85 * TC, gravity=GRAVITY)
    o = olbm.Oracle(p, synth.noisy_density(n, n, n, RHO_BOIL, 0.01, 1234))
    o.step(1)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle", "sample": f"{n}^3 boiling cell, FP64 torch-CPU oracle, {steps} steps"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--tile-x", type=int, default=0)
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--z-chunk", type=int, default=0)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--no-16bit", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true", help="time kernel/tile variants")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.copy_probe:
        import torch
        nbytes = 2 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 10
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes_each_way": nbytes, "ms": round(ms, 4),
                          "gbs_read_plus_write": round(2 * nbytes / ms / 1e6, 1)}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "domain decomposition is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1111_0905_amd import lbm

    lbm.load_library()
    n = args.size
    print(f"bench: generating {n}^3 seeded density field", file=sys.stderr, flush=True)
    rho0 = torch.from_numpy(synth.noisy_density(n, n, n, RHO_BOIL, 0.01, 1234)).cuda().reshape(-1)

    if args.sweep:
        combos = [(0, 32, 16), (2, 64, 16), (0, 64, 8)]
        for kernel, tx, ty in combos:
            for zc in (0, 256, 128):
                r, _ = run_storage(lbm, n, args.storage, args.steps, args.warmup, rho0,
                                   kernel, ty, zc, tx)
                print(json.dumps({"kernel": kernel, "tile": [tx, ty], "z_chunk": zc,
                                  "ms": round(r["ms_per_step"], 4), "mlups": round(r["mlups"], 1),
                                  "gbs": round(r["achieved_gbs"], 1)}), flush=True)
        return

    main_res, tot = run_storage(lbm, n, args.storage, args.steps, args.warmup, rho0,
                                args.kernel, args.tile_y, args.z_chunk, args.tile_x)
    print(f"bench: {args.storage} {main_res['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_16bit:
        for st in ("fp16dev", "bf16dev"):
            r, _ = run_storage(lbm, n, st, args.steps, args.warmup, rho0)
            extra[st] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                         "achieved_gbs": round(r["achieved_gbs"], 1),
                         "frac_of_peak": round(r["achieved_gbs"] / PEAK_HBM_GBS, 4),
                         "speedup_vs_fp32": round(r["mlups"] / main_res["mlups"], 3)}
    cpu = None if args.no_cpu_baseline else cpu_baseline()

    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"boiling convection cell {n}^3, D3Q19 thermal pseudopotential LBM, "
                               f"{args.storage} populations", "nodes": n ** 3,
                   "storage": args.storage, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(main_res["achieved_gbs"], 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(main_res["achieved_gbs"] / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(args.storage, n)},
        "storage_forms": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
