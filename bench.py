"""Benchmark of the harmonic-basis 3PCF hot path on one MI355X.

One step = the whole hot path on one synthetic map already resident in HBM:
build the sky-cell index -> fused multipoles + MFMA contraction over all pivots ->
normalise by the pivots' total weight -> zeta_m copied to the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config nside2048]
Prints one JSON line (progress goes to stderr).
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-multipole updates/s; ζ_m wall time Nside=2048, mixed vs FP64 at 1e-6"
# vector peak: FP64 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz.  Both paths form the
# multipoles with FP64 arithmetic (the mixed path stores them in FP32), so both are judged
# against the FP64 vector peak
PEAK_VALU_TFLOPS = {"mixed": 78.6, "fp64": 78.6}
PEAK_MFMA_TFLOPS = {"mixed": 157.3, "fp64": 78.6}  # dense FP32 / FP64 matrix cores
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


KERNEL_SOURCES = ("z3_multipoles.hip", "z3_device.h")  # the kernel and its device helpers
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
    ap.add_argument("--nside", type=int, default=0,
                    help="run the chosen HEALPix workload's recipe (field, bins, m) at this resolution instead")
    ap.add_argument("--m-max", type=int, default=-1, help="override the workload's largest multipole")
    ap.add_argument("--maps", type=int, default=0,
                    help="override the workload's number of maps (HEALPix and cap workloads)")
    ap.add_argument("--pivot-order", default="ring", choices=["ring", "random"],
                    help="approximate search: pivots in HEALPix RING order or in a seeded random order")
    ap.add_argument("--batch-shape", default="",
                    help="W,T: fix the MFMA many-map kernel's block shape (waves, maps per wave), "
                         "which also selects that kernel for any count above 4 maps")
    ap.add_argument("--shard", default="",
                    help="I/N: time one GPU's share of an N-GPU run, index-order pivots [I n/N, (I+1) n/N) "
                         "against the whole neighbour catalogue (one-map exact search)")
    ap.add_argument("--cross", action="store_true",
                    help="multi-field estimator: three correlated fields on the positions, summed over the "
                         "cyclic permutations of (pivot; b1, b2) fields (one-map workloads)")
    ap.add_argument("--exclude-self", action="store_true",
                    help="leave out the k = j terms of the diagonal (one-map exact search only)")
    ap.add_argument("--save-zeta", default="", help="write the zeta_m of each precision to this .npz")
    ap.add_argument("--adjoint", action="store_true",
                    help="each step also back-propagates L = sum |zeta - t|^2 (random targets) to the field")
    ap.add_argument("--graph", action="store_true",
                    help="with --adjoint: positions fixed, index built once; each step replays one captured HIP "
                         "graph (new values, forward of all maps, adjoint)")
    ap.add_argument("--fd-check", type=int, default=0,
                    help="with --adjoint: check the gradient at this many random (map, pixel) entries against "
                         "central differences of the FP64 forward (after the timed steps)")
    ap.add_argument("--cpu-sample", type=int, default=-1, help="oracle pivots (-1: automatic, 0: skip)")
    ap.add_argument("--hist", type=int, default=0, metavar="N_PHI",
                    help="angular-histogram estimator with N_PHI angular bins (one-map exact search on the "
                         "sky; --m-max up to N_PHI/2 - 1)")
    ap.add_argument("--fftlog", type=int, default=0, metavar="NMODELS",
                    help="FFTLog modelling workload instead of the estimator: A_0, A_1, A_2 of NMODELS "
                         "line-of-sight kernels (N = 256, k in [1e-6, 100], 512 chi points, 64 angles)")
    ap.add_argument("--with-4096", default="auto", choices=["auto", "on", "off"],
                    help="after the timed steps, one step of the Nside 4096 map (exact and approximate search, "
                         "both precisions) as a nested record; auto: with the default Nside 2048 run")
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
              "final all-reduce of zeta, which this program does not run; use --gpus 1", file=sys.stderr)
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

    if args.fftlog > 0:
        fftlog_bench(args, z3, torch)
        return

    cfg = CONFIGS[args.config]
    if args.nside > 0:
        if cfg.kind != "healpix":
            sys.exit("--nside needs a HEALPix workload")
        cfg = dataclasses.replace(cfg, n_or_nside=args.nside, name=f"{cfg.name}@nside{args.nside}")
    if args.m_max >= 0:
        cfg = dataclasses.replace(cfg, m_max=args.m_max, name=f"{cfg.name}@m{args.m_max}")
    if args.maps > 0:
        if cfg.kind == "plane":
            sys.exit("--maps needs a sky workload")
        cfg = dataclasses.replace(cfg, nmaps=args.maps, name=f"{cfg.name}@maps{args.maps}")
    if cfg.kind == "plane" and (args.approx or args.adjoint or args.cross or args.graph):
        print("the plane workload runs the one-map estimator only", file=sys.stderr)
        sys.exit(2)
    if args.hist and (cfg.kind != "healpix" and cfg.kind != "cap" or args.approx or args.adjoint or args.cross
                      or args.exclude_self or args.graph or cfg.nmaps > 1):
        print("--hist runs the one-map exact search on a sky workload", file=sys.stderr)
        sys.exit(2)
    if (args.exclude_self or args.cross) and (args.approx or args.adjoint or cfg.nmaps > 1):
        print("--exclude-self and --cross apply to the one-map exact search only", file=sys.stderr)
        sys.exit(2)
    if args.exclude_self and args.cross:
        print("--exclude-self and --cross are separate options", file=sys.stderr)
        sys.exit(2)
    self_pairs = not args.exclude_self
    shard = None
    if args.shard:
        si, sn = (int(t) for t in args.shard.split("/"))
        if not (0 <= si < sn) or args.approx or args.adjoint or args.cross or cfg.nmaps > 1:
            sys.exit("--shard I/N needs 0 <= I < N and the one-map exact search")
        shard = (si, sn)
    t0 = time.time()
    xyz = make_positions(cfg, device="cuda")
    if cfg.nmaps > 1:
        x = torch.stack([make_values(cfg, xyz, seed=s) for s in range(cfg.nmaps)])
    else:
        x = make_values(cfg, xyz, seed=0)
    x3 = None
    if args.cross:
        # three correlated fields (as for redshift bins of one sky): x0, x0 + x1 / 2, x0 - 0.3 x2
        x1, x2 = make_values(cfg, xyz, seed=1), make_values(cfg, xyz, seed=2)
        x3 = torch.stack([x, x + 0.5 * x1, x - 0.3 * x2])
        del x1, x2
    nbr = None
    if args.approx:
        from synth import degrade_ring
        if cfg.kind != "healpix":
            sys.exit("--approx needs a HEALPix workload")
        nxyz, nx_, nw = degrade_ring(cfg.n_or_nside, x)
        nbr = (nxyz, nx_, nw)
        if args.pivot_order == "random":
            # the library sorts each pivot chunk by the index's bands; this order tests that
            perm = torch.randperm(xyz.shape[1], generator=torch.Generator().manual_seed(11)).to(xyz.device)
            xyz, x = xyz[:, perm].contiguous(), x[perm].contiguous()
            del perm
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

    if args.graph and not args.adjoint:
        sys.exit("--graph needs --adjoint")
    graphs = {}
    last = {}

    shape = tuple(int(v) for v in args.batch_shape.split(",")) if args.batch_shape else None

    def fix_shape(idx):
        if shape:
            idx.set_batch_shape(*shape)

    def graph_step(prec):
        # index and captured graph built once per precision (outside the timed steps)
        if prec not in graphs:
            idx = z3.Index(xyz, E)
            fix_shape(idx)
            idx.set_values(x)
            z0 = z3.estimate_maps_raw(idx, M, prec) if cfg.nmaps > 1 else z3.estimate_raw(idx, M, prec).unsqueeze(0)
            sw = torch.zeros(1, dtype=torch.float64, device="cuda")
            z3.zeta3._lib.call("z3_pivot_weight_sum", idx.handle, 0, idx.n, z3.zeta3._ptr(sw), z3.zeta3._stream())
            t = targets((z0 / sw).reshape((cfg.nmaps,) + tuple(z0.shape[1:])))
            graphs[prec] = (idx, z3.GraphStep(idx, M, t, prec=prec))
            log(f"[bench] {prec}: graph captured, workspace {graphs[prec][1].workspace_bytes / 2**30:.2f} GiB")
        idx, gs = graphs[prec]
        zt, g = gs.run(x.reshape(cfg.nmaps, n))
        grads.append(float(g.abs().max()))
        last["x"], last["zeta"], last["grad"], last["target"] = x, zt, g, gs.target
        zh = zt.cpu().numpy()
        if cfg.nmaps == 1:
            zh = zh[0]
        return zh[..., 0] + 1j * zh[..., 1], pairs_of(idx, prec)

    def step(prec):
        if args.graph:
            return graph_step(prec)
        zeta = torch.zeros((M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        if args.adjoint:
            idx = z3.Index(xyz, E)
            fix_shape(idx)
            xg = x.clone().requires_grad_(True)
            zt = z3.Zeta3Fn.apply(xg, idx, M, prec)
            loss = ((zt - targets(zt)) ** 2).sum()
            loss.backward()
            grads.append(float(xg.grad.abs().max()))
            last["x"], last["zeta"], last["grad"], last["target"] = x, zt.detach(), xg.grad, targets(zt)
            zh = zt.detach().cpu().numpy()
            npairs = pairs_of(idx, prec)
            idx.free()
            return zh[..., 0] + 1j * zh[..., 1], npairs
        if cfg.nmaps > 1:
            zeta = torch.zeros((cfg.nmaps, M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
            idx = z3.Index(xyz, E)
            fix_shape(idx)
            idx.set_values(x)
            z3.estimate_maps_raw(idx, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
        elif x3 is not None:
            idx = z3.Index(xyz, E)
            idx.set_values(x3)
            z3.estimate_cross_raw(idx, (0, 1, 2), M, prec, True, zeta=zeta, pair_total=pairs, sum_w=sw)
        elif args.hist:
            from synth import phi_boundaries
            idx = z3.Index(xyz, E)
            idx.set_values(x)
            idx.set_phi_bins(phi_boundaries(args.hist))
            z3.estimate_hist_raw(idx, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
        elif nbr is None:
            idx = z3.Index(xyz, E, planar=cfg.kind == "plane")
            idx.set_values(x)
            q0, q1 = (0, idx.n) if shard is None else (shard[0] * idx.n // shard[1], (shard[0] + 1) * idx.n // shard[1])
            z3.estimate_raw(idx, M, prec=prec, p0=q0, p1=q1, zeta=zeta, pair_total=pairs, sum_w=sw,
                            self_pairs=self_pairs)
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
        if args.adjoint and not args.graph:
            # the workload's pair count, once and outside the timed steps (the autograd step
            # does not return it; a counting pass costs ~2/3 of a forward)
            pidx = z3.Index(xyz, E)
            pidx.set_values(x)
            pairs_of(pidx, prec)
            pidx.free()
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
    updates = r["pairs"] * (M + 1) * (3 if args.cross else cfg.nmaps)
    value = updates / r["s_per_step"]
    if args.adjoint:
        log(f"[bench] adjoint: max |dL/dx| {max(grads):.3g}")
    launches_per_step = r["kernel_launches"] / args.steps
    kern_s_per_step = r["kernel_ms_total"] / args.steps / 1e3
    if cfg.nmaps > 4 and (shape or cfg.nmaps > (56 if main_prec == "fp64" else 24)):
        # MFMA many-map kernel (the library's choice above 56 maps on the FP64 path and 24 on
        # the mixed one, or with a fixed block shape): one FMA per (pair, map, harmonic
        # column) is the useful work
        rf_kernel, rf_bound, rf_peak = "k_multipoles_batch", "mfma", PEAK_MFMA_TFLOPS[main_prec]
        rf_flops = 2.0 * (2 * M + 1) * r["pairs"] * cfg.nmaps
        rf_unit_note = "2 (2 m_max + 1) flop per (pair, map)"
    elif args.hist:
        # per pair: separation 3, chord 5 + 2 tests, tangent components 10, sign tests 6,
        # histogram add 1 = 27 flop; per (pivot, bin, angular bin, m): 3 flop of the transform
        # (one step of Clenshaw's recurrence, a multiply-add and a subtraction)
        rf_kernel, rf_bound, rf_peak = "k_multipoles_hist", "alu", PEAK_VALU_TFLOPS["fp64"]
        rf_flops = 27.0 * r["pairs"] + 3.0 * n * cfg.nbins * args.hist * (M + 1)
        rf_unit_note = "27 flop per pair + 3 flop per (pivot, radial bin, angular bin, m)"
    else:
        # one-map kernel, or the register-tiled kernel over groups of maps (three fields, or
        # 3 to 56 / 24 maps), whose pair geometry is shared by the maps of a lane
        rf_kernel = "k_multipoles_maps" if (args.cross or cfg.nmaps > 2) else "k_multipoles"
        rf_bound, rf_peak = "alu", PEAK_VALU_TFLOPS[main_prec]
        rf_flops = FLOPS_PER_UPDATE * updates
        rf_unit_note = f"{FLOPS_PER_UPDATE} flop per pair-multipole update"
    achieved = rf_flops / kern_s_per_step / 1e12 if kern_s_per_step > 0 else None
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
        "dtype": "f64" if main_prec == "fp64" else "f64 multipoles, f32 storage + split-f32 MFMA",
        "data": "synthetic",
        "config": {"workload": cfg.name + ("+approx" if nbr else "") + ("+adjoint" if args.adjoint else "")
                   + ("+random-order" if nbr and args.pivot_order == "random" else "")
                   + (f"+hist{args.hist}" if args.hist else "")
                   + ("+noself" if not self_pairs else "") + ("+cross3" if args.cross else "")
                   + (f"+shard{shard[0]}of{shard[1]}" if shard else ""),
                   "npoints": n, "nmaps": cfg.nmaps, "nbins": cfg.nbins, "m_max": M,
                   **({"r_plane_units": [cfg.theta_min, cfg.theta_max]} if cfg.kind == "plane" else
                      {"theta_arcmin": [cfg.theta_min * 10800 / np.pi, cfg.theta_max * 10800 / np.pi]}),
                   "log_bins": cfg.log_bins, "precision": main_prec, "pairs": r["pairs"]},
        "roofline": {"bound": rf_bound, "kernel": rf_kernel, "achieved": achieved,
                     "peak": rf_peak, "unit": "TFLOP/s", "frac": achieved / rf_peak if achieved else None,
                     "traffic": measured_traffic(cfg.name, main_prec)
                     if rf_kernel == "k_multipoles" and self_pairs and not args.cross and shard is None else None,
                     "traffic_unit": "bytes per launch",
                     "avg_launch_ms": r["kernel_ms_total"] / r["kernel_launches"] if r["kernel_launches"] else None,
                     "launches_per_step": launches_per_step, "flops": rf_unit_note,
                     **({"note": "kernel time is not measurable inside a graph replay"} if not achieved else {})},
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
        out["mixed_vs_fp64_entries"] = entry_errors(res["mixed"]["zeta"], res["fp64"]["zeta"])

    if args.adjoint and args.fd_check > 0:
        out["fd_check"] = fd_check(cfg, xyz, E, M, last, args.fd_check, z3, torch)
        log(f"[bench] fd check: {out['fd_check']}")
    if args.graph:
        out["config"]["graph"] = "index built once; each step = one replay of a captured HIP graph " \
                                 "(value update, forward of all maps, loss gradient, adjoint)"
        out["config"]["workload"] += "+graph"
    if args.save_zeta:
        np.savez(args.save_zeta, **{p: res[p]["zeta"] for p in res})
    out["config"]["inputs_sha256"] = inputs_digest(xyz, x if x3 is None else x3, torch)
    if args.cpu_sample != 0 and cfg.nmaps == 1 and not args.cross and cfg.kind != "plane" and shard is None \
            and not args.hist:
        out["cpu_baseline"] = cpu_baseline(cfg, xyz, x, nbr, E, M, args.cpu_sample, z3, torch, self_pairs)
    plain = (args.config == "nside2048" and args.nside == 0 and args.m_max < 0 and not (
        args.approx or args.adjoint or args.cross or args.exclude_self or shard or args.graph or args.hist))
    if args.with_4096 == "on" or (args.with_4096 == "auto" and plain and args.prec == "both"):
        del xyz, x
        torch.cuda.empty_cache()
        out["nside4096"] = nside4096_record(z3, torch)
    print(json.dumps(out), flush=True)


def inputs_digest(xyz, x, torch):
    """SHA-256 of the workload's inputs as the library receives them (positions, then values,
    FP64 bytes in catalogue order), streamed from the device in slices after the timed steps,
    so that a record names exactly the data it measured."""
    import hashlib
    h = hashlib.sha256()
    for t in (xyz, x):
        flat = t.reshape(-1)
        for s in range(0, flat.numel(), 1 << 24):
            h.update(flat[s:s + (1 << 24)].to(torch.float64).cpu().numpy().tobytes())
    return h.hexdigest()


def entry_errors(test, ref):
    """Error of the mixed path against FP64 per (m, b1, b2) and component: |test - ref| / |ref|,
    with entries where |ref| < 1e-3 max_m |ref| flagged as cancellation-limited (their
    relative error measures the rounding of a near-zero sum, not the path); per m the largest
    relative error over the well-conditioned entries, and the worst entries overall.  Several
    maps ([map][m][b1][b2]): every map's entries, per m the worst map."""
    if ref.ndim == 3:
        test, ref = test[None], ref[None]
    rows = []
    per_m = [None] * ref.shape[1]
    ncanc = 0
    for k in range(ref.shape[0]):
        for m in range(ref.shape[1]):
            r = np.stack([ref[k, m].real, ref[k, m].imag], -1)
            t = np.stack([test[k, m].real, test[k, m].imag], -1)
            scale = np.abs(r).max()
            d = np.abs(t - r)
            canc = np.abs(r) < 1e-3 * scale
            if m == 0:
                canc[..., 1] = True  # Im zeta_0 is 0 by construction
            b1, b2 = np.meshgrid(np.arange(r.shape[0]), np.arange(r.shape[1]), indexing="ij")
            for c in (0, 1):
                cm = canc[..., c]
                ncanc += int(cm.sum())
                rel = np.where(cm, np.nan, d[..., c] / np.where(cm, 1.0, np.abs(r[..., c])))
                for i, j in zip(b1[~cm], b2[~cm]):
                    rows.append((float(rel[i, j]), k, m, int(i), int(j), "re" if c == 0 else "im"))
            good = ~canc
            if good.any():
                e = float((d[good] / np.abs(r[good])).max())
                per_m[m] = e if per_m[m] is None else max(per_m[m], e)
    rel_all = np.array([q[0] for q in rows])
    worst = sorted(rows, reverse=True)[:5]
    return {"entries": int(ref.size * 2), "cancellation_limited": ncanc,
            "rule": "cancellation-limited: |zeta64| < 1e-3 of the largest |zeta64| of that m (and Im zeta_0)",
            "max_rel_err": float(rel_all.max()), "median_rel_err": float(np.median(rel_all)),
            "p99_rel_err": float(np.percentile(rel_all, 99)), "max_rel_err_per_m": per_m,
            "worst": [{"rel_err": q[0], **({"map": q[1]} if ref.shape[0] > 1 else {}), "m": q[2], "b1": q[3],
                       "b2": q[4], "part": q[5]} for q in worst]}


def nside4096_record(z3, torch):
    """One step of the full-sky Nside 4096 workload (201,326,592 pixels, 20 log bins 2'-120',
    m <= 10) in each precision: exact search, and the approximate search (the same pivots
    against the Nside 2048 averaged neighbour map).  Each step builds the index, runs the fused
    estimator, normalises and copies zeta to the host, as the timed Nside 2048 steps do."""
    from synth import CONFIGS, degrade_ring, make_positions, make_values
    cfg = CONFIGS["nside4096"]
    M = cfg.m_max
    E = cfg.edges_chord2()
    t0 = time.time()
    xyz = make_positions(cfg, device="cuda")
    x = make_values(cfg, xyz, seed=0)
    nxyz, nx_, nw = degrade_ring(cfg.n_or_nside, x)
    torch.cuda.synchronize()
    log(f"[bench] nside4096 inputs generated in {time.time() - t0:.1f}s")
    rec = {"workload": "nside4096", "npoints": int(xyz.shape[1]), "nbins": cfg.nbins, "m_max": M,
           "theta_arcmin": [cfg.theta_min * 10800 / np.pi, cfg.theta_max * 10800 / np.pi],
           "steps": 1, "warmup": 0, "note": "one step per (search, precision) after the Nside 2048 steps"}
    for search in ("exact", "approx"):
        sub = {}
        zs = {}
        for prec in ("fp64", "mixed"):
            zeta = torch.zeros((M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
            pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
            sw = torch.zeros(1, dtype=torch.float64, device="cuda")
            z3.profile_read(reset=True)
            z3.profile_enable(True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            if search == "exact":
                idx = z3.Index(xyz, E)
                idx.set_values(x)
                z3.estimate_raw(idx, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
            else:
                idx = z3.Index(nxyz, E, weights=nw)
                idx.set_values(nx_)
                z3.estimate_pivots_raw(idx, xyz, x, None, M, prec=prec, zeta=zeta, pair_total=pairs, sum_w=sw)
            z3.zeta3._lib.call("z3_finalize", 1, M, cfg.nbins, z3.zeta3._ptr(zeta), z3.zeta3._ptr(sw),
                               z3.zeta3._stream())
            zh = zeta.cpu().numpy()
            npairs = int(pairs.item())
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            z3.profile_enable(False)
            launches, kms = z3.profile_read(reset=True)
            idx.free()
            zs[prec] = zh[..., 0] + 1j * zh[..., 1]
            updates = npairs * (M + 1)
            ach = FLOPS_PER_UPDATE * updates / (kms / 1e3) / 1e12 if kms > 0 else None
            sub[prec] = {"zeta_wall_s": dt, "pairs": npairs, "updates_per_s": updates / dt,
                         "k_multipoles_ms": kms, "launches": launches,
                         "roofline_frac": ach / PEAK_VALU_TFLOPS[prec] if ach else None,
                         "achieved_tflops": ach}
            log(f"[bench] nside4096 {search} {prec}: {dt:.2f} s, {npairs} pairs, k_multipoles {kms:.0f} ms "
                f"in {launches} launches")
        e = err_m(zs["mixed"], zs["fp64"])
        sub["mixed_vs_fp64_err_m"] = e
        sub["mixed_vs_fp64_err_max"] = max(e)
        sub["pairs_equal"] = sub["fp64"]["pairs"] == sub["mixed"]["pairs"]
        sub["speedup_mixed_vs_fp64"] = sub["fp64"]["zeta_wall_s"] / sub["mixed"]["zeta_wall_s"]
        rec[search] = sub
        if search == "exact":
            zexact = zs["fp64"]
        else:
            sub["approx_vs_exact_err_m"] = err_m(zs["fp64"], zexact)
    del xyz, x, nxyz, nx_, nw
    torch.cuda.empty_cache()
    return rec


def fd_check(cfg, xyz, E, M, last, k, z3, torch):
    """Gradient of L = sum (zeta - t)^2 at k random (map, pixel) entries against central
    differences of the FP64 forward.  zeta is a quadratic function of any single value x_i
    (x_i enters as a pivot value and through the multipoles of its neighbours' bins), so
    the central difference of zeta is exact up to rounding for any step h; the adjoint
    computes sum_G G . dzeta/dx_i with G = 2 (zeta - t) at the evaluated forward."""
    x = last["x"].reshape(cfg.nmaps, -1)
    n = x.shape[1]
    G = (2.0 * (last["zeta"] - last["target"])).reshape(cfg.nmaps, M + 1, cfg.nbins, cfg.nbins, 2)
    grad = last["grad"].reshape(cfg.nmaps, n)
    rng = np.random.default_rng(4_000_000)
    maps = rng.integers(0, cfg.nmaps, size=k)
    pix = rng.choice(n, size=k, replace=False)
    idx = z3.Index(xyz, E)
    idx.set_values(x[0].contiguous())
    sw = torch.zeros(1, dtype=torch.float64, device="cuda")
    z3.zeta3._lib.call("z3_pivot_weight_sum", idx.handle, 0, n, z3.zeta3._ptr(sw), z3.zeta3._stream())
    scale = 1.0 / float(sw.item())
    fd, ad = [], []
    t0 = time.perf_counter()
    for s_, i in zip(maps, pix):
        xm = x[s_].clone()
        h = 32.0 * float(xm.std())
        zs = []
        for sign in (1.0, -1.0):
            xp = xm.clone()
            xp[i] += sign * h
            idx.update_values(xp)
            zs.append(z3.estimate_raw(idx, M, "fp64") * scale)
        dz = (zs[0] - zs[1]) / (2.0 * h)
        fd.append(float((G[s_] * dz).sum()))
        ad.append(float(grad[s_, i]))
    idx.free()
    fd, ad = np.array(fd), np.array(ad)
    err = np.abs(ad - fd) / np.abs(fd).max()
    return {"entries": k, "max_rel_err": float(err.max()), "median_rel_err": float(np.median(err)),
            "max_abs_grad": float(np.abs(fd).max()), "seconds": time.perf_counter() - t0,
            "note": "relative to the largest sampled gradient; FP64 forward differences, exact for the "
                    "quadratic dependence of zeta on one value"}


FFTLOG_SETTINGS = dict(N=256, k_min=1e-6, k_max=100.0, nchi=512, chi_min=1e-4, chi_max=60.0, ntheta=64,
                       theta_min=0.002, theta_max=0.2)
FFTLOG_NU = (-0.3, -1.3, -1.3, -0.3)  # biases of the (0,0), (1,1), (1,-1), (2,0) factors


def fftlog_bench(args, z3, torch):
    """A_0, A_1, A_2 of a batch of line-of-sight kernels through z3_fftlog_a_functions.  The
    dominant kernel is the product of the angle factor's s1 >= 0 half with the Hankel matrix of
    the chi integrals (three launches per pass, one per function): 8 ntheta (N + 1) (N/2 + 1)
    flop per launch and model (complex FP64 multiply-adds)."""
    import hashlib
    from synth import fftlog_inputs
    S = FFTLOG_SETTINGS
    nm = args.fftlog
    Pk, F, theta, _, _ = fftlog_inputs(N=S["N"], k_min=S["k_min"], k_max=S["k_max"], nchi=S["nchi"],
                                       chi_min=S["chi_min"], chi_max=S["chi_max"], nmodels=nm, ntheta=S["ntheta"],
                                       theta_min=S["theta_min"], theta_max=S["theta_max"], seed=11)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Pk_d, F_d, th_d = dev(Pk), dev(F), dev(theta)
    ws = torch.empty(z3.fftlog_workspace_size(S["N"], S["nchi"], S["ntheta"], nm), dtype=torch.uint8, device="cuda")
    out = torch.empty((nm, 3, S["ntheta"], S["ntheta"]), dtype=torch.float64, device="cuda")

    def run():
        z3.fftlog_a_functions(Pk_d, S["k_min"], S["k_max"], FFTLOG_NU, F_d, S["chi_min"], S["chi_max"], th_d,
                              workspace=ws, out=out)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    z3.profile_read(reset=True)
    z3.profile_enable(True)
    t = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    launches, kms = z3.profile_read(reset=True)
    z3.profile_enable(False)
    ns = S["N"] + 1
    flops_launch = 8.0 * S["ntheta"] * ns * (S["N"] // 2 + 1) * nm
    kern_s = kms / max(launches, 1) / 1e3
    achieved = flops_launch / kern_s / 1e12 if kern_s > 0 else None
    total_flops = nm * 3 * (4.0 * ns * S["nchi"] + 8.0 * S["ntheta"] * ns * (S["N"] // 2 + 1)
                            + 4.0 * S["ntheta"] ** 2 * ns)
    log(f"[bench] fftlog: {nm} models in {dt * 1e3:.2f} ms/step; k_cgemm<2> {kms / max(launches, 1):.3f} ms "
        f"x {launches / args.steps:.0f} per step ({achieved:.1f} TFLOP/s)")
    # oracle on a bounded sample of the models, and GPU parity on the same models
    from oracle import fftlog
    from synth import log_grid
    chi = log_grid(S["chi_min"], S["chi_max"], S["nchi"])
    got = out.cpu().numpy()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    ns_cpu, t_cpu, err = 0, 0.0, 0.0
    while ns_cpu < nm and t_cpu < 10.0:
        t0 = time.perf_counter()
        ref = fftlog.a_functions(Pk, S["k_min"], S["k_max"], chi, F[ns_cpu], theta, *FFTLOG_NU).real
        t_cpu += time.perf_counter() - t0
        err = max(err, float(np.abs(got[ns_cpu] - ref).max() / np.abs(ref).max()))
        ns_cpu += 1
    log(f"[bench] fftlog oracle: {ns_cpu} models in {t_cpu:.2f}s, GPU max-normalised error {err:.2e}")
    rec = {
        "metric": "FFTLog A-function sets/s (A_0, A_1, A_2 on a 64 x 64 angle grid)",
        "value": nm / dt,
        "unit": "models/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"fftlog N={S['N']} k=[1e-6,100] nchi={S['nchi']} ntheta={S['ntheta']} "
                               f"models={nm}", "nu": list(FFTLOG_NU), **S, "nmodels": nm,
                   "total_flops_per_step": total_flops,
                   "inputs_sha256": hashlib.sha256(Pk.tobytes() + F.tobytes() + theta.tobytes()).hexdigest()},
        "roofline": {"bound": "mfma", "kernel": "k_cgemm<2>", "achieved": achieved,
                     "peak": PEAK_MFMA_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_MFMA_TFLOPS["fp64"] if achieved else None, "traffic": None,
                     "avg_launch_ms": kms / max(launches, 1), "launches_per_step": launches / args.steps,
                     "flops": "8 ntheta (N+1) (N/2+1) flop per product (omega U1) H and model"},
        "cpu_baseline": {"value": ns_cpu / t_cpu, "unit": "models/s", "cores": threads, "kind": "oracle",
                         "sample": f"the first {ns_cpu} models, one oracle call each (NumPy, BLAS threads)",
                         "seconds": t_cpu, "gpu_max_err_on_sample": err},
    }
    print(json.dumps(rec), flush=True)


def cpu_baseline(cfg, xyz, x, nbr, E, M, nsample, z3, torch, self_pairs=True):
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
        return cpu.estimate(xyz_h[:, sel], nbr_h[0], nbr_h[2], nbr_h[1], E, M, w_h[sel], x_h[sel], nthreads=threads,
                            self_pairs=self_pairs)

    def timed(k):
        t = time.perf_counter()
        zo_, po_ = oracle(order[p0:p0 + k])
        return zo_, po_, time.perf_counter() - t

    # sample size: whole rounds of the oracle's 1,024-pivot blocks over its threads (full
    # occupancy), grown until one call takes >= 10 s; the oracle's neighbour-grid set-up, part
    # of every call, is timed on its own and left out of the rate
    round_ = 1024 * threads
    if nsample < 0:
        rounds = 1
        while True:
            k = min(n - p0, rounds * round_)
            zo, po, dt = timed(k)
            log(f"[bench] cpu_baseline: {k} pivots ({rounds} round(s) of {threads} x 1024) in {dt:.2f}s")
            if dt >= 10.0 or k >= n - p0:
                break
            rounds = max(rounds + 1, int(rounds * min(8.0, 11.0 / max(dt, 1e-3))))
        nsample = k
    else:
        log(f"[bench] cpu_baseline: oracle on {nsample} pivots x {threads} threads")
        zo, po, dt = timed(nsample)
    t_setup = cpu.setup_seconds(nbr_h[0], nbr_h[2], nbr_h[1], E, M)
    log(f"[bench] cpu_baseline: oracle grid set-up {t_setup:.2f}s of the {dt:.2f}s call")
    parity = {}
    for gp in ("fp64", "mixed"):
        zeta = torch.zeros((M + 1, cfg.nbins, cfg.nbins, 2), dtype=torch.float64, device="cuda")
        pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
        sw = torch.zeros(1, dtype=torch.float64, device="cuda")
        if nbr is None:
            z3.estimate_raw(idx, M, prec=gp, p0=p0, p1=p0 + nsample, zeta=zeta, pair_total=pairs, sum_w=sw,
                            self_pairs=self_pairs)
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
    return {"value": po * (M + 1) / max(dt - t_setup, 1e-9), "unit": "pair-multipole updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{nsample} contiguous pivots ({nsample // round_} full rounds of {threads} threads x 1024-pivot "
                      f"blocks) from position {p0} of the {cfg.name} map against all {len(nbr_h[1])} neighbours; "
                      f"rate over the call minus the oracle's grid set-up",
            "seconds": dt, "grid_setup_seconds": t_setup, "value_including_setup": po * (M + 1) / dt,
            "cpu_model": cpu_model(), "gpu_parity_on_sample": parity}


if __name__ == "__main__":
    main()
