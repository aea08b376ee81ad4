"""Throughput of the thermal pseudopotential D3Q19 step on one MI355X.

Workload: the 512^3 boiling convection cell in FP32 (walls at z, periodic x, y;
Ra = 1e7, Pr = 9, nu = 0.0165; mean density such that the bottom layer of the
hydrostatic liquid column lies past the liquid spinodal), the paper's
resolution (L = 512, Table 1).  A step is one full lattice update
(every step of the hot path: moments, pseudopotential and thermal forces,
both BGK collisions with the counter-term, streaming and the walls) with the
populations resident in HBM.

Prints one JSON line: MLUPS, ms per step, the roofline of the step kernel
(algorithmic bytes = one read and one write of each node's stored
populations: 2 x 152 B in FP32, 2 x 80 B in the 16-bit forms) against the
8 TB/s of the data sheet and against references timed in the same
process with the library's plain streaming kernels (a 16-byte-per-lane copy
of 8 GiB each way, and the step's 19-row read/write pattern without its
arithmetic, with 400 MiB rows and with the state's own rows), the
FP16/BF16-deviation storage forms beside it, and the FP64
CPU oracle timed on a bounded sample on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + achieved HBM GB/s (% of peak), FP32 vs FP16-storage, 512^3 boiling"
PEAK_HBM_GBS = 8000.0
# bytes of one node's populations in one buffer (read once, written once per step)
NODE_BYTES = {"fp64": 19 * 16, "fp32": 19 * 8, "fp16dev": 18 * 4 + 8, "bf16dev": 18 * 4 + 8}

RA = 1e7                               # Rayleigh number of the boiling cell (Table 1 order)


def workload_params(lbm, n, storage, kernel=0, tile_y=0, z_chunk=0, tile_x=0):
    """The boiling convection cell of side n: T_c = 0.08, T_d = 0.95 T_c,
    T_u = 0.85 T_c, nu = 0.0165, Pr = 9 in the liquid, gravity from Ra, mean
    density 0.12 below that of the hydrostatic liquid column whose bottom
    layer sits on the liquid spinodal."""
    from paper_1111_0905_amd import experiments
    rho = experiments.boiling_density(n, RA)
    return experiments.cell_params(n, rho, RA, storage, kernel=kernel, tile_x=tile_x,
                                   tile_y=tile_y, z_chunk=z_chunk)


def seeded_density(n, rho_mean):
    import synth
    return synth.noisy_density(n, n, n, rho_mean, 0.01, 1234)


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
    bpn = 2 * NODE_BYTES[storage]
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
    """SHA-256 of the kernel sources' code: comments and blank space are
    dropped first, so that a change of wording does not disown the counter
    runs of an unchanged kernel."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1111_0905_amd", "csrc", "*.hip")) +
                    glob.glob(os.path.join(ROOT, "paper_1111_0905_amd", "csrc", "*.hpp"))):
        with open(p) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(storage, n):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on this very kernel source and workload (else None)."""
    path = os.path.join(ROOT, "profiles", f"step_{storage}_{n}cubed_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha256") != source_hash():
        return None
    return d["traffic_bytes_per_launch"]


def bandwidth_references(lbm, n, gib=8, reps=5):
    """HBM references timed in this process with the library's plain
    streaming kernels: the 16-byte-per-lane copy of `gib` GiB each way (plain
    and non-temporal; the faster counts) and the step's row pattern without
    arithmetic (19 rows read and written per thread), once with rows of 400
    MiB (7.4 GiB each way) and once per storage form with rows of the n^3
    state's own moving rows (n^3 x 8 B for FP32, n^3 x 4 B for the 16-bit
    forms, whose rest row is n^3 x 8 B) at the state's row pitch, the
    footprint the step streams.
    GB/s of reads plus writes."""
    import torch
    nbytes = gib << 30
    state_row = {"fp32": n ** 3 * 8, "fp16dev": n ** 3 * 4, "bf16dev": n ** 3 * 4}
    # rows of the state lie row_pitch words apart (the node count rounded up to
    # 16384, plus 1024: the library's layout)
    pitch = -(-n ** 3 // 16384) * 16384 + 1024
    state_stride = {"fp32": pitch * 8, "fp16dev": pitch * 4, "bf16dev": pitch * 4}
    a = torch.ones(max(nbytes, 19 * max(state_stride.values())) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    copy = {}
    for nt in (False, True):
        ms = timed(lambda: lbm.lbm_stream_copy(a, b, nbytes, nt))
        copy["nontemporal" if nt else "plain"] = 2 * nbytes / ms / 1e6
    row = 400 << 20
    ms = timed(lambda: lbm.lbm_stream_rows(a, b, 19, row, row))
    rows19 = 2 * 19 * row / ms / 1e6
    rows19_state = {}
    for st, rb in state_row.items():
        if st == "bf16dev":               # the same rows as fp16dev
            rows19_state[st] = rows19_state["fp16dev"]
            continue
        rb -= rb % 8                       # the row kernel moves 8-byte words
        ms = timed(lambda: lbm.lbm_stream_rows(a, b, 19, state_stride[st], rb))
        rows19_state[st] = 2 * 19 * rb / ms / 1e6
    del a, b
    torch.cuda.empty_cache()
    return {"copy_gbs": max(copy.values()), "copy_plain_gbs": copy["plain"],
            "copy_nontemporal_gbs": copy["nontemporal"], "rows19_gbs": rows19,
            "rows19_state_gbs": rows19_state}


def diagnostics_timing(lbm, n, reps=5):
    """Wall time of one step followed by one FP64 diagnostic on a new state
    (so rho, E and psi are recomputed once), for lbm_moments and lbm_nusselt,
    FP32 and FP16 storage; one JSON line each."""
    import torch
    rho_mean = workload_params(lbm, n, "fp32").rho_ref
    rho0 = lbm.lbm_seeded_density(n, n, n, 1234, rho_mean, 0.01).reshape(-1)
    for st in ("fp32", "fp16dev"):
        lat = lbm.Lattice(workload_params(lbm, n, st), rho0)
        lat.step(2)
        for what in ("moments", "nusselt"):
            fn = (lambda: lat.moments()) if what == "moments" else (lambda: lat.nusselt())
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                lat.step(1)
                fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            print(json.dumps({"storage": st, "diagnostic": what, "nodes": n ** 3,
                              "ms_step_plus_diagnostic": round(ms, 3)}), flush=True)
        del lat
        torch.cuda.empty_cache()


def cpu_baseline(seconds=15.0, n=64, max_steps=None):
    """FP64 oracle on the host, n^3 sample of the same physics, stepped for
    about `seconds` (or max_steps) after one warm-up step."""
    import torch
    from oracle import lbm as olbm
    threads = os.cpu_count() or 1
    torch.set_num_threads(threads)
    from paper_1111_0905_amd import lbm
    w = workload_params(lbm, 512, "fp32")      # physics of the full-size cell
    p = olbm.Params(n, n, n, tau_nu=w.tau_nu, tau_kappa=w.tau_kappa, G=w.G, T_d=w.T_d,
                    T_u=w.T_u, gravity=w.gravity, c_v=w.c_v, rho_kappa=w.rho_kappa,
                    T_lat=w.T_lat)
    o = olbm.Oracle(p, seeded_density(n, w.rho_ref))
    o.step(1)
    steps = 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0 < seconds) if max_steps is None else (steps < max_steps):
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
    ap.add_argument("--no-references", action="store_true",
                    help="skip the copy and row-pattern bandwidth references")
    ap.add_argument("--sweep", action="store_true", help="time kernel/tile variants")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the library's plain 2 GiB copy (calibrates HBM byte counters)")
    ap.add_argument("--diagnostics", action="store_true",
                    help="only time one step plus each FP64 diagnostic (lbm_moments, lbm_nusselt) "
                         "at --size, FP32 and FP16 storage, one JSON line each")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 CPU oracle at 32^3, 64^3 (100 steps) and 128^3 "
                         "(20 steps), one JSON line each")
    args = ap.parse_args()

    if args.oracle_timing:
        for n, steps in ((32, 100), (64, 100), (128, 20)):
            print(json.dumps(cpu_baseline(n=n, max_steps=steps)), flush=True)
        return

    if args.copy_probe:
        # the library's plain 16-byte copy of 2 GiB (calibrates the HBM byte
        # counters: FETCH_SIZE and WRITE_SIZE of a copy of known size)
        import torch
        from paper_1111_0905_amd import lbm
        lbm.load_library()
        nbytes = 2 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            lbm.lbm_stream_copy(src, dst, nbytes)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 10
        for _ in range(reps):
            lbm.lbm_stream_copy(src, dst, nbytes)
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
    from paper_1111_0905_amd import lbm

    lbm.load_library()
    n = args.size
    if args.diagnostics:
        diagnostics_timing(lbm, n)
        return
    print(f"bench: generating {n}^3 seeded density field", file=sys.stderr, flush=True)
    rho_mean = workload_params(lbm, n, "fp32").rho_ref
    # the same field as seeded_density (bit for bit), generated on the device
    rho0 = lbm.lbm_seeded_density(n, n, n, 1234, rho_mean, 0.01).reshape(-1)

    if args.sweep:
        combos = [(3, 128, 4), (3, 64, 8), (3, 32, 16), (3, 32, 8), (0, 32, 16), (0, 64, 8),
                  (2, 64, 16), (2, 64, 8)]
        for kernel, tx, ty in combos:
            for zc in (0,):
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
                         # on 2 x 76 B per node (all 38 populations in 16 bits)
                         "frac_of_peak_152B": round(152 * n ** 3 / (r["ms_per_step"] * 1e-3) / 1e9
                                                    / PEAK_HBM_GBS, 4),
                         "speedup_vs_fp32": round(r["mlups"] / main_res["mlups"], 3),
                         "traffic": measured_traffic(st, n)}
    refs = None if args.no_references else bandwidth_references(lbm, n)
    if refs:
        rs = refs["rows19_state_gbs"]
        print(f"bench: copy {refs['copy_gbs']:.0f} GB/s, 19-row pattern {refs['rows19_gbs']:.0f} GB/s "
              f"(400 MiB rows), {rs['fp32']:.0f} GB/s (FP32 state rows), {rs['fp16dev']:.0f} GB/s "
              "(16-bit state rows)", file=sys.stderr, flush=True)
        for st, r in extra.items():
            r["frac_of_copy"] = round(r["achieved_gbs"] / refs["copy_gbs"], 4)
            r["frac_of_rows19_state"] = round(r["achieved_gbs"] / rs[st], 4)
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
                     "traffic": measured_traffic(args.storage, n),
                     "copy_gbs": round(refs["copy_gbs"], 1) if refs else None,
                     "frac_of_copy": round(main_res["achieved_gbs"] / refs["copy_gbs"], 4) if refs else None,
                     "rows19_gbs": round(refs["rows19_gbs"], 1) if refs else None,
                     "frac_of_rows19": round(main_res["achieved_gbs"] / refs["rows19_gbs"], 4) if refs else None,
                     "rows19_state_gbs": round(refs["rows19_state_gbs"][args.storage], 1)
                     if refs and args.storage in refs["rows19_state_gbs"] else None,
                     "frac_of_rows19_state": round(main_res["achieved_gbs"]
                                                   / refs["rows19_state_gbs"][args.storage], 4)
                     if refs and args.storage in refs["rows19_state_gbs"] else None},
        "bandwidth_references": refs,
        "storage_forms": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
