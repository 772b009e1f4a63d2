#!/usr/bin/env python3
"""Benchmark of the bispectrum-multipole estimator on one MI355X.

Metric: (k1, mu, t) bins x (l, m) multipoles estimated per second for one
N_g = 256 field (40 k1 x 20 mu x 10 t bins, 16 multipoles = 128 000 values per
estimate), float32 path; the float64 path is timed beside it for the
FP32/FP64 speedup.  One step = one complete estimate (forward FFT, ring FFTs,
triple products, binning) of a field already resident in HBM.

Prints ONE JSON line.  Extra keys: per-stage times, the float64 path, the
roofline of the dominant kernel (the triple-product contraction), the
float64 CPU oracle timed on a bounded sample, and the error per multipole
against stored oracle values when they exist.

  python bench.py [--steps K] [--warmup W] [--ng 256|128] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "triangle bins x (l,m) estimated/sec at N_g=256; FP32-batched vs FP64 speedup"
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_FP64_TFLOPS = 78.6
WORKLOADS = {
    256: dict(n_k1=40, k1_min=1.0, k1_max=256 / 3, n_mu=20, n_t=10, n_s=-2.0),
    128: dict(n_k1=20, k1_min=1.0, k1_max=128 / 3, n_mu=10, n_t=10, n_s=-2.0),
    512: dict(n_k1=60, k1_min=1.0, k1_max=512 / 3, n_mu=20, n_t=15, n_s=-1.5),
}
# uneven batch: 24 fields at N_g = 64, 24 at 96, 16 at 128 (seeds 0..63), one graph launch
BATCHED = [(64, 24), (96, 24), (128, 16)]


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("bk_kernels.hpp", "bk_fft.hpp", "bk_tables.hpp", "bk_tables.cpp", "bk_api.hip"):
        with open(os.path.join(ROOT, "paper_2405_14513_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(ng):
    """HBM bytes per K3 launch from a committed rocprofv3 --pmc summary, or None
    if absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"k3_contract_traffic_ng{ng}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_path(bk, torch, binning, prec, field, steps, warmup, tune=True):
    """Times one estimate per step.  The timed region runs `steps` estimates
    launched kernel by kernel with hipEvents between the stages, on torch's
    current stream, with no host synchronisation inside; the library averages
    the stage times over them.  The graph-replayed estimate (bk_estimate) is
    timed the same way beside it."""
    est = bk.Estimator(binning, prec=prec)
    stream = torch.cuda.current_stream().cuda_stream
    est.load(field, stream)
    choices = est.autotune(stream) if tune else None  # untimed, like plan creation
    for _ in range(warmup):
        est.estimate(stream)
        est.estimate_timed(stream)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        est.estimate_timed(stream)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    stages = est.stage_times()  # mean over the timed region's estimates (the last 32 at most)
    start.record()
    for _ in range(steps):
        est.estimate(stream)
    end.record()
    torch.cuda.synchronize()
    ms_graph = start.elapsed_time(end) / steps
    B = est.multipoles()[0]
    info = est.info()
    info["tiles"] = choices
    info["graph_ms"] = ms_graph
    info["stages_averaged"] = min(steps, 32)
    est.close()
    return ms, stages, B, info


def read_k2_traffic(ng):
    """HBM bytes per estimate of the ring-sum launches from a committed
    rocprofv3 --pmc summary, or None (absent or other kernel sources)."""
    path = os.path.join(ROOT, "profiles", f"k2_ring_traffic_ng{ng}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_estimate"])
    except (KeyError, ValueError):
        return None


def per_bin_relative(B, ref, floor=1e-3):
    """Largest |B - B_ref| / |B_ref| over the bins with |B_ref| > floor * max |B_ref|, per multipole."""
    import numpy as np

    out = []
    for j in range(ref.shape[0]):
        ok = ~np.isnan(ref[j])
        r = ref[j][ok]
        b = B[j][ok]
        big = np.abs(r) > floor * np.max(np.abs(r))
        out.append(float(np.max(np.abs(b[big] - r[big]) / np.abs(r[big]))))
    return out


def cpu_baseline(delta64, ng, wl, info):
    """The float64 oracle on every m-th plane triple, projected to one estimate."""
    import numpy as np

    from oracle.estimator import stream_plane_triples
    from oracle.geometry import Binning, make_rings, make_sides, plane_triples, triangle_counts

    try:
        from threadpoolctl import threadpool_info

        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = 1
    b = Binning(ng, wl["n_k1"], wl["k1_min"], wl["k1_max"], wl["n_mu"], wl["n_t"])
    stride = 97 if ng >= 256 else 23
    t0 = time.perf_counter()
    rings = make_rings(ng)
    ntri = triangle_counts(rings)
    sides = make_sides(rings, b)
    t_setup = time.perf_counter() - t0
    triples = plane_triples(int(np.ceil(b.k1_max)))
    sample = triples[::stride]
    t0 = time.perf_counter()
    _, _, _, n_visited = stream_plane_triples(delta64, b, rings, ntri, sides, sample)
    t_sample = time.perf_counter() - t0
    total = 2 * info["combinations"] - info["self_partnered"]  # the oracle visits both n -> -n partners
    t_full = t_setup + t_sample * total / max(n_visited, 1)
    n_values = b.n_bins * len(b.lms())
    return {
        "value": n_values / t_full,
        "unit": "bin-multipoles/s",
        "cores": int(cores),
        "kind": "oracle",
        "projected": True,
        "sample": (f"PROJECTED from a sample: float64 oracle (numpy FFT + BLAS contraction) on every {stride}th of "
                   f"{len(triples)} plane triples, {n_visited} of {int(total)} combinations (both n -> -n partners "
                   f"counted, as the oracle visits them) in {t_sample:.1f} s, plus {t_setup:.1f} s of ring/N_tri "
                   f"setup; projected full estimate {t_full:.0f} s"),
    }


def run_batched(args, np, torch, bk, FieldRecipe, make_field):
    """All fields of the uneven batch in one hipGraph launch (one plan per N_g)."""
    stream = torch.cuda.current_stream().cuda_stream
    plans, tensors = [], []
    seed = 0
    n_values = 0
    for ng, count in BATCHED:
        binning = bk.make_binning(ng, 20, 1.0, ng / 3, 10, 10)
        f = np.stack([make_field(FieldRecipe(ng, n_s=-2.0, f_ng=0.5, beta=0.5, seed=seed + i)) for i in range(count)])
        seed += count
        t = torch.from_numpy(f.astype(np.float32)).cuda()
        plan = bk.bk_plan_create(binning, bk.BK_F32, 0, count)
        bk.bk_load_grid(plan, t.data_ptr(), bk.BK_F32, count, True, stream)
        bk.bk_plan_autotune(plan, stream)  # untimed; the graph captures the tuned tiles
        plans.append(plan)
        tensors.append(t)
        n_values += count * 20 * 10 * 10 * 16
    group = bk.bk_group_create(plans)
    for _ in range(args.warmup):
        bk.bk_group_estimate(group, stream)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        bk.bk_group_estimate(group, stream)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    B = [bk.bk_get_multipoles(p, c) for p, (_, c) in zip(plans, BATCHED)]
    finite = all(np.isfinite(b).any() for b in B)
    # the first N_g = 96 field (seed 24) against its stored float64 oracle values
    err96 = None
    gold = os.path.join(ROOT, "tests", "golden", "oracle_ng96.npz")
    if os.path.exists(gold):
        g = np.load(gold)
        i96 = [ng for ng, _ in BATCHED].index(96)
        ref = g["B"].reshape(16, -1)
        Bf = B[i96][0].reshape(16, -1)
        ok = ~np.isnan(ref)
        if np.array_equal(np.isnan(Bf), ~ok):
            err96 = max(float(np.max(np.abs(Bf[j][ok[j]] - ref[j][ok[j]])) / np.max(np.abs(ref[j][ok[j]])))
                        for j in range(16))
    n_fields = sum(c for _, c in BATCHED)
    out = {
        "metric": "bin-multipoles estimated/sec, uneven batch of 64 fields in one graph launch",
        "value": n_values / (ms * 1e-3),
        "unit": "bin-multipoles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("uneven batch: 24 fields at N_g=64, 24 at 96, 16 at 128 (seeds 0..63, P ~ k^-2, f_NG 0.5, "
                         "beta 0.5); per field 20 k1 shells on [1, N_g/3), 10 mu x 10 t bins, 16 multipoles"),
            "fields_per_step": n_fields,
        },
        "realisations_per_s": n_fields / (ms * 1e-3),
        "outputs_finite": bool(finite),
        "max_error_vs_oracle_ng96_seed24": err96,
    }
    bk.bk_group_destroy(group)
    for p in plans:
        bk.bk_plan_destroy(p)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ng", type=int, default=256, choices=sorted(WORKLOADS))
    ap.add_argument("--batched", action="store_true",
                    help="time the uneven batch (24 x N_g=64, 24 x 96, 16 x 128, float32) as one graph launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile choices")
    ap.add_argument("--all-l", action="store_true",
                    help="every l <= 6 (odd l from Im S: twice the contraction's matrix work), not the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this estimator build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_14513_amd import bk
    from synth import FieldRecipe, field_digest, make_field

    if args.batched:
        run_batched(args, np, torch, bk, FieldRecipe, make_field)
        return
    ng = args.ng
    wl = WORKLOADS[ng]
    binning = bk.make_binning(ng, wl["n_k1"], wl["k1_min"], wl["k1_max"], wl["n_mu"], wl["n_t"],
                              even_l_only=0 if args.all_l else 1)
    n_lm = 28 if args.all_l else 16  # l <= 6, m <= 6: every l, or even l only
    recipe = FieldRecipe(ng, n_s=wl["n_s"], f_ng=0.5, beta=0.5, seed=0)
    delta64 = make_field(recipe)
    digest = field_digest(delta64)
    f32 = torch.from_numpy(delta64.astype(np.float32)).cuda()
    f64 = torch.from_numpy(delta64).cuda()

    ms32, st32, B32, info = time_path(bk, torch, binning, bk.BK_F32, f32, args.steps, args.warmup,
                                      not args.no_autotune)
    n_values = wl["n_k1"] * wl["n_mu"] * wl["n_t"] * n_lm
    out = {
        "metric": METRIC,
        "value": n_values / (ms32 * 1e-3),
        "unit": "bin-multipoles/s",
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
            "workload": (f"N_g={ng} periodic box (cell 1), field g + 0.5 (g^2 - <g^2>) with P ~ k^{wl['n_s']:g} and Kaiser "
                         f"beta 0.5 along z, seed 0; {wl['n_k1']} linear k1 shells on [1, N_g/3), "
                         f"{wl['n_mu']} mu x {wl['n_t']} t bins, {n_lm} multipoles l <= 6, m <= 6"
                         + (" (every l; odd l from Im S)" if args.all_l else "")),
            "ng": ng,
            "bins": [wl["n_k1"], wl["n_mu"], wl["n_t"]],
            "n_lm": n_lm,
            "fields_per_step": 1,
            "input": "float32 grid resident in HBM",
        },
    }
    stage_names = ["fft3d", "ring_fft", "triple_products", "binning"]
    k3_ms = float(st32[2])
    out["stage_ms"] = {k: float(st32[i]) for i, k in enumerate(stage_names)}
    out["graph_ms_per_step"] = info["graph_ms"]
    # Re(D_A D_C D_B): 2 FMAs per (combination, x_perp) with D_A D_C reused; Im S (every l) 2 more
    per_term = 8.0 if args.all_l else 4.0
    flops = info["useful_terms"] * per_term
    achieved = flops / (k3_ms * 1e-3) / 1e12
    traffic = None if args.all_l else read_traffic(ng)
    out["roofline"] = {
        "kernel": "k3_contract_kernel<float>",
        "bound": "mfma",
        "achieved": achieved,
        "peak": PEAK_FP32_MFMA_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
        "traffic": traffic,
        "algorithmic_flops_per_launch": flops,
        "dense_flops_per_launch": info["dense_terms"] * per_term,
        "avg_launch_ms": k3_ms,
        "launches_averaged": info["stages_averaged"],
    }
    # counter evidence (rocprofv3 --pmc summaries committed under profiles/)
    d_bytes = info["d_elems_per_field"] * 8.0  # complex64 D
    if traffic is not None:
        out["roofline"]["k3_traffic_over_d_bytes"] = traffic / d_bytes
    # K2 algorithmic bytes: D written once plus the Delta planes read once
    k2_alg = d_bytes + (int(np.ceil(wl["k1_max"])) + 1) * ng * ng * 8.0
    k2_ms = float(st32[1])
    out["k2_ring_sums"] = {
        "algorithmic_bytes": k2_alg,
        "achieved_GBps": k2_alg / (k2_ms * 1e-3) / 1e9,
        "frac_of_8TBps": k2_alg / (k2_ms * 1e-3) / 8e12,
        "traffic": read_k2_traffic(ng) if not args.all_l else None,
    }
    out["plan"] = {k: info[k] for k in ("combinations", "work_items", "sides", "rings", "plane_triples")}
    out["plan"]["tiles"] = info["tiles"]  # [FFT lines, ring-sum columns, slots per chunk]
    # first-level estimates per second: every combination and its n -> -n partner (one S serves both)
    first_level = 2 * info["combinations"] - info["self_partnered"]
    out["first_level_combinations_per_s"] = first_level / (ms32 * 1e-3)
    if not args.no_fp64:
        ms64, st64, B64, info64 = time_path(bk, torch, binning, bk.BK_F64, f64, args.steps, args.warmup,
                                            not args.no_autotune)
        out["fp64"] = {
            "ms_per_step": ms64,
            "graph_ms_per_step": info64["graph_ms"],
            "value": n_values / (ms64 * 1e-3),
            "stage_ms": {k: float(st64[i]) for i, k in enumerate(stage_names)},
            "tiles": info64["tiles"],
        }
        out["fp32_vs_fp64_speedup"] = ms64 / ms32
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_ng{ng}.npz")
    if os.path.exists(gold) and not args.all_l:
        g = np.load(gold)
        if str(g["digest"]) == digest:
            ref = g["B"].reshape(16, -1)
            errs, rel = {}, {}
            for name, B in (("f32", B32), ("f64", B64 if not args.no_fp64 else None)):
                if B is None:
                    continue
                Bf = B.reshape(16, -1)
                ok = ~np.isnan(ref)
                e = [float(np.max(np.abs(Bf[j][ok[j]] - ref[j][ok[j]])) / np.max(np.abs(ref[j][ok[j]])))
                     for j in range(16)]
                errs[name] = e
                rel[name] = per_bin_relative(Bf, ref)
            out["error_per_multipole_vs_oracle"] = errs
            out["per_bin_relative_error_vs_oracle"] = {
                "definition": "max |B - B_oracle| / |B_oracle| over bins with |B_oracle| > 1e-3 max |B_oracle|",
                **rel,
            }
    if args.copy_calibration:
        # a plain streaming kernel of known size: y = 2 x over 1 GiB reads 1 GiB and writes 1 GiB
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": x.numel() * 4, "write": y.numel() * 4}
        del x, y
    if not args.no_cpu_baseline and not args.all_l:
        out["cpu_baseline"] = cpu_baseline(delta64, ng, wl, info)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
