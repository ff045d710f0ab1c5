"""Benchmark of the harmonic-basis 3PCF hot path on one MI355X.

One step = the whole hot path on one synthetic map already resident in HBM:
build the sky-cell index -> fused multipoles + MFMA contraction over all pivots ->
normalise by the pivots' total weight -> zeta_m copied to the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config nside2048]
Prints one JSON line (progress goes to stderr).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-multipole updates/s; ζ_m wall time Nside=2048, mixed vs FP64 at 1e-6"
PEAK_VALU_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (non-packed FP32 or FP64 FMA)
FLOPS_PER_UPDATE = 12.5  # algorithmic flops per (pair, m) at m_max = 10: 10 per m + ~35 per pair / 11


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


KERNEL_SOURCES = ("z3_multipoles.hip", "z3_device.h", "z3_internal.h")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_multipoles_traffic.json")


def kernel_source_hash():
    """sha256 over the sources k_multipoles is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2408_16847_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(cfg_name, prec):
    """HBM bytes per k_multipoles launch from the committed rocprofv3 counter passes, if they
    were taken on this exact kernel source, workload and precision; otherwise None."""
    try:
        rec = json.load(open(TRAFFIC_JSON))
        digest = kernel_source_hash()
    except OSError:
        return None
    if rec.get("source_sha256") != digest:
        return None
    if rec.get("workload") != cfg_name or rec.get("precision") != prec:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def _counter_rows(path, counter, name_part):
    import csv
    with open(path, newline="") as f:
        return [float(r["Counter_Value"]) for r in csv.DictReader(f)
                if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]]


def write_traffic_json(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, cfg_name, prec):
    """Turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE passes (KiB per dispatch) over k_multipoles
    and over the plain copy of `--copy-calibration` into bytes per launch, each counter scaled
    so that it reads the copy's known size."""
    copy_bytes = 8 << 28
    cf = max(_counter_rows(copy_fetch_csv, "FETCH_SIZE", "copyBuffer"))
    cw = max(_counter_rows(copy_write_csv, "WRITE_SIZE", "copyBuffer"))
    fs, ws = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    f = _counter_rows(fetch_csv, "FETCH_SIZE", "k_multipoles<")
    w = _counter_rows(write_csv, "WRITE_SIZE", "k_multipoles<")
    if not f or not w:
        sys.exit("no k_multipoles dispatch in the counter files")
    rec = {"kernel": "k_multipoles", "source_sha256": kernel_source_hash(), "workload": cfg_name,
           "precision": prec, "dispatches": len(f),
           "fetch_bytes_per_launch": sum(f) / len(f) * 1024.0 * fs,
           "write_bytes_per_launch": sum(w) / len(w) * 1024.0 * ws,
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
           "note": "FETCH_SIZE/WRITE_SIZE KiB averaged over the dispatches (one launch per pivot chunk), scaled by the "
                   "plain-copy calibration (2 GiB read, 2 GiB written)"}
    with open(TRAFFIC_JSON, "w") as fo:
        json.dump(rec, fo, indent=1)
        fo.write("\n")
    print(json.dumps(rec))


def err_m(test, ref):
    if ref.ndim == 4:  # several maps: the worst map per m
        return [max(v) for v in zip(*[err_m(t, r) for t, r in zip(test, ref)])]
    out = []
    for m in range(ref.shape[0]):
        r = np.concatenate([ref[m].real.ravel(), ref[m].imag.ravel()])
        t = np.concatenate([test[m].real.ravel(), test[m].imag.ravel()])
        den = np.abs(r).max()
        out.append(float(np.abs(t - r).max() / (den if den > 0 else 1.0)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="nside2048")
    ap.add_argument("--prec", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--approx", action="store_true",
                    help="approximate search: neighbours from the Nside/2 averaged map, all pivots kept")
    ap.add_argument("--save-zeta", default="", help="write the zeta_m of each precision to this .npz")
    ap.add_argument("--adjoint", action="store_true",
                    help="each step also back-propagates L = sum |zeta - t|^2 (random targets) to the field")
    ap.add_argument("--cpu-sample", type=int, default=-1, help="oracle pivots (-1: automatic, 0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter calibration)")
    ap.add_argument("--traffic-json", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the k_multipoles HBM traffic record from rocprofv3 counter CSVs (no GPU needed)")
    args = ap.parse_args()

    if args.traffic_json:
        write_traffic_json(*args.traffic_json, args.config, "mixed" if args.prec == "both" else args.prec)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the estimator's pivot sum would shard over GPUs with one "
              "final all-reduce of zeta, which this build does not run; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2408_16847_amd as z3
    from synth import CONFIGS, make_positions, make_values

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 28  # 2 GiB of FP64
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}))
        return

    cfg = CONFIGS[args.config]
    t0 = time.time()
    xyz = make_positions(cfg, device="cuda")
    if cfg.nmaps > 1:
        x = torch.stack([make_values(cfg, xyz, seed=s) for s in range(cfg.nmaps)])
    else:
        x = make_values(cfg, xyz, seed=0)
    nbr = None
    if args.approx:
        from synth import degrade_ring
        if cfg.kind != "healpix":
            sys.exit("--approx needs a HEALPix workload")
        nxyz, nx_, nw = degrade_ring(cfg.n_or_nside, x)
        nbr = (nxyz, nx_, nw)
    torch.cuda.synchronize()
    log(f"[bench] inputs {cfg.name}{' approx' if nbr else ''}: n={xyz.shape[1]} generated in "
        f"{time.time() - t0:.1f}s; delta min {float(x.min()):.3g} max {float(x.max()):.3g}")
    E = cfg.edges_chord2()
    M = cfg.m_max
    n = xyz.shape[1]

    grads = []
    _tgt = {}
    _pairs = {}

    def targets(zt):
        # random FP64 targets t = N(0,1) * rms(zeta_m) per entry (seeded), fixed across steps
        if "t" not in _tgt:
            rng = np.random.default_rng(3_000_000)
            rms = zt.detach().pow(2).mean(dim=tuple(range(zt.dim() - 3, zt.dim())), keepdim=True).sqrt()
            _tgt["t"] = torch.from_numpy(rng.normal(size=tuple(zt.shape))).cuda() * rms
        return _tgt["t"]

    def pairs_of(idx, prec):
        # pair count of the workload, measured once outside the timed steps' arithmetic
        if prec not in _pairs:
            pt = torch.zeros(1, dtype=torch.int64, device="cuda")
            z3.accumulate(idx, 0, 0, idx.n, prec=prec, want_a=False, pair_total=pt)
            _pairs[prec] = int(pt.item())
        return _pairs[prec]

    def step(prec):
        zeta = torch.zeros((M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        if args.adjoint:
            idx = z3.Index(xyz, E)
            xg = x.clone().requires_grad_(True)
            zt = z3.Zeta3Fn.apply(xg, idx, M, prec)
            loss = ((zt - targets(zt)) ** 2).sum()
            loss.backward()
            grads.append(float(xg.grad.abs().max()))
            zh = zt.detach().cpu().numpy()
            npairs = pairs_of(idx, prec)
            idx.free()
            return zh[..., 0] + 1j * zh[..., 1], npairs
        if cfg.nmaps > 1:
            zeta = torch.zeros((cfg.nmaps, M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
            idx = z3.Index(xyz, E)
            idx.set_values(x)
            z3.estimate_maps_raw(idx, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
        elif nbr is None:
            idx = z3.Index(xyz, E)
            idx.set_values(x)
            z3.estimate_raw(idx, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
        else:
            idx = z3.Index(nbr[0], E, weights=nbr[2])
            idx.set_values(nbr[1])
            z3.estimate_pivots_raw(idx, xyz, x, None, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
        z3.zeta3._lib.call("z3_finalize", cfg.nmaps, M, cfg.nbins, z3.zeta3._ptr(zeta), z3.zeta3._ptr(sw),
                           z3.zeta3._stream())
        zh = zeta.cpu().numpy()
        npairs = int(pairs.item())
        idx.free()
        return zh[..., 0] + 1j * zh[..., 1], npairs

    precs = ["fp64", "mixed"] if args.prec == "both" else [args.prec]
    res = {}
    for prec in precs:
        for w in range(args.warmup):
            step(prec)
            log(f"[bench] {prec} warmup {w + 1}/{args.warmup} done")
        z3.profile_read(reset=True)
        z3.profile_enable(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in range(args.steps):
            zeta, npairs = step(prec)
            log(f"[bench] {prec} step {s + 1}/{args.steps} done")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        z3.profile_enable(False)
        launches, kms = z3.profile_read(reset=True)
        res[prec] = {"zeta": zeta, "pairs": npairs, "s_per_step": dt, "kernel_ms_total": kms,
                     "kernel_launches": launches}
        log(f"[bench] {prec}: {dt * 1e3:.1f} ms/step, pairs {npairs}, "
            f"k_multipoles {kms / max(launches, 1):.2f} ms x {launches / args.steps:.0f} per step")

    main_prec = "mixed" if "mixed" in res else "fp64"
    r = res[main_prec]
    updates = r["pairs"] * (M + 1) * cfg.nmaps
    value = updates / r["s_per_step"]
    if args.adjoint:
        log(f"[bench] adjoint: max |dL/dx| {max(grads):.3g}")
    launches_per_step = r["kernel_launches"] / args.steps
    kern_s_per_step = r["kernel_ms_total"] / args.steps / 1e3
    achieved = FLOPS_PER_UPDATE * updates / kern_s_per_step / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-multipole updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["s_per_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f64 geometry + f32 multipoles/MFMA",
        "data": "synthetic",
        "config": {"workload": cfg.name + ("+approx" if nbr else "") + ("+adjoint" if args.adjoint else ""),
                   "npoints": n, "nmaps": cfg.nmaps, "nbins": cfg.nbins, "m_max": M,
                   "theta_arcmin": [cfg.theta_min * 10800 / np.pi, cfg.theta_max * 10800 / np.pi],
                   "log_bins": cfg.log_bins, "precision": main_prec, "pairs": r["pairs"]},
        "roofline": {"bound": "alu", "kernel": "k_multipoles", "achieved": achieved,
                     "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                     "traffic": measured_traffic(cfg.name, main_prec),
                     "traffic_unit": "bytes per launch", "avg_launch_ms": r["kernel_ms_total"] / max(r["kernel_launches"], 1),
                     "launches_per_step": launches_per_step, "flops_per_update": FLOPS_PER_UPDATE},
    }
    for prec in res:
        out[f"zeta_wall_ms_{prec}"] = res[prec]["s_per_step"] * 1e3
        out[f"updates_per_s_{prec}"] = res[prec]["pairs"] * (M + 1) * cfg.nmaps / res[prec]["s_per_step"]
    if "fp64" in res and "mixed" in res:
        e = err_m(res["mixed"]["zeta"], res["fp64"]["zeta"])
        out["mixed_vs_fp64_err_m"] = e
        out["mixed_vs_fp64_err_max"] = max(e)
        out["speedup_mixed_vs_fp64"] = res["fp64"]["s_per_step"] / res["mixed"]["s_per_step"]
        out["pairs_equal"] = res["fp64"]["pairs"] == res["mixed"]["pairs"]

    if args.save_zeta:
        np.savez(args.save_zeta, **{p: res[p]["zeta"] for p in res})
    if args.cpu_sample != 0 and cfg.nmaps == 1:
        out["cpu_baseline"] = cpu_baseline(cfg, xyz, x, nbr, E, M, args.cpu_sample, z3, torch)
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, xyz, x, nbr, E, M, nsample, z3, torch):
    """Time the FP64 C oracle on a contiguous range of pivots against the full neighbour
    catalogue, and check the GPU path on the same pivots."""
    from oracle import cpu
    n = xyz.shape[1]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    if nbr is None:
        idx = z3.Index(xyz, E)
        idx.set_values(x)
        order = idx.perm().cpu().numpy()  # GPU pivot ranges are in index order
        nbr_h = (xyz.cpu().numpy(), x.cpu().numpy(), np.ones(n))
    else:
        idx = z3.Index(nbr[0], E, weights=nbr[2])
        idx.set_values(nbr[1])
        order = np.arange(n)  # external pivots keep the caller's order
        nbr_h = (nbr[0].cpu().numpy(), nbr[1].cpu().numpy(), nbr[2].cpu().numpy())
    xyz_h = xyz.cpu().numpy()
    x_h = x.cpu().numpy()
    w_h = np.ones(n)
    p0 = n // 3

    def oracle(sel):
        return cpu.estimate(xyz_h[:, sel], nbr_h[0], nbr_h[2], nbr_h[1], E, M, w_h[sel], x_h[sel], nthreads=threads)

    # size the sample to ~15 s of oracle work: one call with a single pivot measures the
    # oracle's fixed cost (its own O(N) grid build); its pair rate is measured on 320 pivots,
    # then again on ~2 s worth of pivots (small calls under-use the threads)
    if nsample < 0:
        t = time.perf_counter()
        oracle(order[p0:p0 + 1])
        t_fixed = time.perf_counter() - t
        k, rate = 320, 0.0
        for target in (None, 2.0):
            if target is not None:
                k = int(min(n - p0, max(320, target * rate / per_pivot)))
            t = time.perf_counter()
            _, pk = oracle(order[p0:p0 + k])
            rate = pk / max(time.perf_counter() - t - t_fixed, 1e-3)
            per_pivot = max(pk / k, 1.0)
            log(f"[bench] cpu_baseline calibration: fixed {t_fixed:.2f}s, {k} pivots at {rate:.3g} pairs/s")
        nsample = int(min(n - p0, max(320, 15.0 * rate / per_pivot)))
    sel = order[p0:p0 + nsample]
    log(f"[bench] cpu_baseline: oracle on {nsample} pivots x {threads} threads")
    t = time.perf_counter()
    zo, po = oracle(sel)
    dt = time.perf_counter() - t
    parity = {}
    for gp in ("fp64", "mixed"):
        zeta = torch.zeros((M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        if nbr is None:
            z3.estimate_raw(idx, M, prec=gp, p0=p0, p1=p0 + nsample, zeta=zeta, pair_total=pairs, sum_w=sw)
        else:
            z3.estimate_pivots_raw(idx, xyz, x, None, M, prec=gp, p0=p0, p1=p0 + nsample, zeta=zeta,
                                   pair_total=pairs, sum_w=sw)
        zg = (zeta / sw).cpu().numpy()
        zg = zg[..., 0] + 1j * zg[..., 1]
        e = err_m(zg, zo)
        parity[gp] = {"pairs_equal": po == int(pairs.item()), "err_m_max": max(e)}
        log(f"[bench] cpu_baseline: {dt:.1f}s; {gp} on the sample: pairs oracle {po} gpu {int(pairs.item())}, "
            f"err_m max {max(e):.2e}")
    idx.free()
    return {"value": po * (M + 1) / dt, "unit": "pair-multipole updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsample} contiguous pivots from position {p0} of the {cfg.name} map against all "
                      f"{len(nbr_h[1])} neighbours (includes the oracle's O(N) grid build)",
            "seconds": dt, "cpu_model": cpu_model(),
            "gpu_parity_on_sample": parity}


if __name__ == "__main__":
    main()
