"""Benchmark: B-hat^T N^-1 B-hat elements/s on one MI355X.

A step is one pass of the whole device path on one synthetic problem:
tabulate the beam and prior kernels (each with its unique-block evaluation),
then write the D-hat blocks and contract B-hat^T N^-1 B-hat (one launch, the
combined call).  Grid construction is host work done once per resolution and
is timed separately (grid_setup_s).  Inputs are resident in device memory
before the timed region.

Default workload: lmax = 3000, k = 8 (13.0M pixels, 1,013,648 stored 64x64
blocks), Gaussian beam FWHM 3 pixels cut at 3 FWHM, prior d_l = (l+1)^2,
N^-1 = log-normal scan-stripe pattern with 20% of the sky masked.

value = stored B^T N^-1 B elements / step time in plain FP64 (the paper's
arithmetic); the mixed-precision modes (split BF16 with 6 or 3 products, FP32
MFMA) are timed the same way and reported under "modes", each with its error
against the FP64 oracle ("gate": max |GPU - oracle| / M_J on sampled block
rows, M_J the largest oracle value of block-row J) and its speed relative to
FP64.  The oracle runs only in the cpu_baseline leg: it computes the sampled
block-rows there (that is the baseline's timed work), and the same rows are
then compared with every mode's last timed output.

With --config batch32 a step is one launch of the captured graph that contracts
all 32 problems of the batched workload (lmax 256/512/1024/2048; FP32 MFMA
with FP64 accumulation across contraction tiles first, then split BF16x6 and
plain FP64; 172 GB of output), one batch per mode, the first reported as
value; the beam kernels are tabulated before the timed region and the schedule
and tile shape are autotuned first.

With --op conv a step is one pixel-domain convolution g = B-hat f (FP64) of
the configuration's grid and beam.  With --op two_hop a step tabulates the beam
kernel and samples B^T N^-1 B on the two-hop pattern (every nonzero block of
the product), in the first of --modes.  With --op two_grid a step tabulates
the beam kernel between the configuration's grid Y_1 and an auxiliary grid Y_2
(--lmax2, default twice lmax) and samples B^T N_2^-1 B with N_2^-1 on Y_2.
With --op sht a step is one synthesis and one analysis at L = lmax.  With
--op factor the FP64 operators come from one combined call before the timed
region, and a step factors every tile's diagonal block of
D-hat + B^T N^-1 B (Cholesky) and applies the block-Jacobi solve once.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config lmax3000|batch32]
                       [--op btnb|conv|two_hop|two_grid|sht|factor] [--lmax2 L]
                       [--modes fp64,bf16x6,fp32,bf16x3]
                       [--no-cpu-baseline] [--no-batch-compare]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "B^T N^-1 B elements/s at lmax=3000: FP64 vs split-BF16 MFMA at <=1e-6 rel err"
HEADLINE = "fp64"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}     # TFLOP/s, dense
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6}                   # MFMA products per term
BOUND = {"fp64": 1e-10, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 2.0 ** -15}  # gate each mode is held to
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x6": "bf16", "bf16x3": "bf16"}
HBM_PEAK = 8000.0                                                              # GB/s
FP64_VECTOR = 78.6     # TFLOP/s: FP64 FMA on the vector ALUs (256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz)
KERNEL_NAME = {"fp64": "k_class_f64<false>", "fp32": "k_class_f32<false>", "bf16x3": "k_class_bf16<2, false>",
               "bf16x6": "k_class_bf16<3, false>"}
BATCH_KERNEL = {"fp64": "k_batch_f64", "fp32": "k_batch_f32", "bf16x6": "k_batch_bf16<3>",
                "bf16x3": "k_batch_bf16<2>"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="lmax3000")
    ap.add_argument("--op", default="btnb", choices=["btnb", "conv", "two_hop", "two_grid", "sht", "factor"],
                    help="btnb: the D-hat / B-hat^T N^-1 B-hat step (default); conv: the pixel-domain "
                         "convolution g = B-hat f; two_hop: B^T N^-1 B on every nonzero block of the product; "
                         "two_grid: B^T N_2^-1 B with N_2^-1 on an auxiliary grid (--lmax2, default twice); "
                         "sht: spherical harmonic synthesis + analysis on the grid (L = lmax) and the degrade "
                         "of Eq. 14 onto a grid of half the band limit")
    ap.add_argument("--lmax2", type=int, default=0, help="band limit of the auxiliary grid for --op two_grid")
    ap.add_argument("--modes", default=None,
                    help="precision modes, the first is reported as value (default fp64,bf16x6,fp32,bf16x3; "
                         "for --config batch32 fp32,bf16x6,fp64)")
    ap.add_argument("--separate", action="store_true",
                    help="sample D-hat and B^T N^-1 B with the two separate calls (default: the combined "
                         "call, one launch)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="tabulate each step's kernels on the main stream, after the previous step (default: on a "
                         "second stream, while the previous step's sampling launch runs)")
    ap.add_argument("--no-batch-compare", action="store_true",
                    help="skip the untimed comparison of the contraction alone in the class-kernel grid and "
                         "as a one-problem persistent batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-seconds-1t", type=float, default=6.0,
                    help="budget of the single-BLAS-thread oracle run")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one plain device-to-device copy of BYTES bytes (a reference "
                         "kernel of known traffic for HBM counter runs)")
    args = ap.parse_args()
    if args.modes is None:
        args.modes = "fp32,bf16x6,fp64" if args.config == "batch32" else "fp64,bf16x6,fp32,bf16x3"
    return args


def kernels_hash(source="kernels.hip"):
    src = os.path.join(ROOT, "paper_1504_04653_amd", "csrc", source)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def recorded_traffic(mode, config, source="kernels.hip"):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current source of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.md")
    if not os.path.exists(path):
        return None
    h = kernels_hash(source)
    for line in open(path):
        m = re.match(r"\|\s*(\S+)\s*\|\s*(\S+)\s*\|\s*(\S+)\s*\|\s*([0-9.eE+]+)\s*\|\s*([0-9.eE+]+)\s*\|", line)
        if m and m.group(1) == mode and m.group(2) == config and m.group(3) == h:
            return float(m.group(4)) + float(m.group(5))
    return None


def host_info():
    """Host cores, CPU model and the BLAS library numpy calls (vendor,
    version, threads)."""
    info = {"nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if blas:
            info["blas"] = {"vendor": blas[0].get("internal_api"), "version": blas[0].get("version"),
                            "threads": int(blas[0].get("num_threads", 1))}
    except Exception:  # pragma: no cover
        pass
    return info


def blas_threads(info):
    return int(info.get("blas", {}).get("threads", 1))


def gate(C, ref, rows):
    """max |C - ref| / M_J over the blocks compared, M_J the largest |ref| of
    block-row J (rows[n] = J of block n); infinite if anything is not finite."""
    if not (np.isfinite(C).all() and np.isfinite(ref).all()):
        return float("inf")
    mj = {}
    for n, J in enumerate(rows):
        mj[J] = max(mj.get(J, 0.0), float(np.abs(ref[n]).max()))
    worst = 0.0
    for n, J in enumerate(rows):
        d = float(np.abs(C[n] - ref[n]).max())
        worst = max(worst, d / mj[J] if mj[J] > 0 else d)
    return worst


def error_summary(C, ref, rows):
    """Gate plus the per-element |C - ref| / max(|ref|, 1e-8 M_J) median / p99 / max."""
    mj = {}
    for n, J in enumerate(rows):
        mj[J] = max(mj.get(J, 0.0), float(np.abs(ref[n]).max()))
    scale = np.array([mj[J] for J in rows])[:, None, None]
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.abs(C - ref) / np.maximum(np.maximum(np.abs(ref), 1e-8 * scale), 1e-300)
    return {"gate": gate(C, ref, rows), "median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
            "max": float(np.max(rel))}


def sampled_rows(tiles, n_random, seed):
    """Block-rows J to check: the first tile of the two polar bands, of the two
    equatorial bands and of up to four bands whose tile count differs from a
    neighbour's, then random tiles (in that order)."""
    tiles = np.asarray(tiles)
    t0 = np.concatenate([[0], np.cumsum(tiles)[:-1]])
    nb = len(tiles)
    nh = nb // 2
    special = list(dict.fromkeys([0, 1, nb - 2, nb - 1]))
    ntrans = 0
    for b in range(nb):
        i, south = divmod(b, 2)
        nbrs = [2 * (i - 1) + south] if i > 0 else []
        nbrs.append(2 * (i + 1) + south if i < nh - 1 else 2 * i + 1 - south)
        if b not in special and ntrans < 4 and any(tiles[x] != tiles[b] for x in nbrs):
            special.append(b)
            ntrans += 1
    rows = []
    for b in special:
        if int(t0[b]) not in rows:
            rows.append(int(t0[b]))
    rng = np.random.default_rng(seed)
    ntiles = int(tiles.sum())
    target = min(ntiles, len(rows) + n_random)
    while len(rows) < target:
        J = int(rng.integers(ntiles))
        if J not in rows:
            rows.append(J)
    return rows


def row_blocks(blk_ptr, blk_col, rows):
    """Library stored-block indices and (J, K) pairs of the given rows."""
    idx, pairs = [], []
    for J in rows:
        for n in range(int(blk_ptr[J]), int(blk_ptr[J + 1])):
            idx.append(n)
            pairs.append((J, int(blk_col[n])))
    return np.asarray(idx, dtype=np.int64), pairs


def cpu_baseline(cfg, g, budget_s, budget_1t, sampled):
    """The oracle as it stands, timed on the sampled block-rows of the same
    workload (in order, until the budget is spent; unique blocks evaluated on
    first use inside the timed region), first with numpy's BLAS threads, then
    on one BLAS thread.  The rows it computed are then compared with every
    mode's GPU output of those rows (sampled = {"rows", "pairs", "modes":
    {mode: {"C": blocks, "D": blocks or None}}})."""
    from oracle import grid as G
    from oracle import operators as O
    from workloads import synth as S
    info = host_info()
    og = G.make_grid(cfg.lmax, cfg.k)
    ring, _, _, phi = og.pixel_coords()
    ninv = S.ninv_for(cfg, og.theta[ring], phi)
    b_l, R = S.gaussian_beam(cfg.lmax, og.npix, cfg.fwhm_pix)
    rows, pairs = sampled["rows"], sampled["pairs"]
    # the library's stored-block rows must list the oracle's neighbours K >= J
    layout_ok = all([K for J2, K in pairs if J2 == J] == [K for K in og.tile_neighbours(J) if K >= J]
                    for J in rows)
    by_row = {}
    for n, (J, K) in enumerate(pairs):
        by_row.setdefault(J, []).append((n, K))

    def run(budget):
        op = O.LocalOperator(og, b_l, R)
        done, out = [], []
        t0 = time.perf_counter()
        for J in rows:
            if done and time.perf_counter() - t0 >= budget:
                break
            for n, K in by_row[J]:
                out.append(O.btnb_block(op, ninv, J, K))
                done.append(n)
        return time.perf_counter() - t0, done, out

    dt, done, Cref = run(budget_s)
    res = {"value": len(done) * 4096 / dt, "unit": "elements/s", "cores": blas_threads(info), "kind": "oracle",
           "sample": f"{len(set(pairs[n][0] for n in done))} block-rows ({len(done)} stored 64x64 blocks of "
                     f"B^T N^-1 B: polar, equatorial and ratio-transition bands, then random tiles) of the "
                     f"lmax={cfg.lmax} workload, unique blocks evaluated on first use, {dt:.1f} s wall, "
                     f"numpy FP64 with {blas_threads(info)} BLAS threads",
           "host": info, "layout_matches_oracle": bool(layout_ok)}
    if budget_1t > 0:
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"):
                dt1, done1, _ = run(budget_1t)
            res["single_thread"] = {"value": len(done1) * 4096 / dt1, "unit": "elements/s", "cores": 1,
                                    "sample": f"the first {len(done1)} of the same blocks, {dt1:.1f} s wall"}
        except Exception as e:  # pragma: no cover
            res["single_thread"] = {"error": str(e)}
    # the same rows against every mode's last timed output
    Cref = np.stack(Cref)
    jrow = [pairs[n][0] for n in done]
    Dref = None
    gates = {}
    for mode, m in sampled["modes"].items():
        r = {"C": error_summary(m["C"][done], Cref, jrow), "bound": BOUND[mode]}
        if m.get("D") is not None:
            if Dref is None:
                Dref = O.sample_D(og, S.prior(cfg.lmax), None, [pairs[n] for n in done])
            r["D"] = error_summary(m["D"][done], Dref, jrow)
        r["blocks"] = len(done)
        if not layout_ok:
            r["C"]["gate"] = float("inf")          # the blocks compared are not the oracle's
        gates[mode] = r
    return res, gates




def batch_inputs(sp, S):
    """The 32 problems of the batched workload, with library grids shared per lmax."""
    grids, probs = {}, []
    for p in range(32):
        prob = S.batch_problem(p)
        lmax = prob["lmax"]
        if lmax not in grids:
            g = sp.Grid(lmax, 8)
            grids[lmax] = (g, g.pixel_theta_phi())
        g, (th, ph) = grids[lmax]
        b_l, R = S.gaussian_beam(lmax, g.npix, prob["fwhm_pix"])
        probs.append(dict(prob=prob, g=g, b_l=b_l, R=R, ninv=S.ninv_batch(th, ph, prob)))
    return probs


def cpu_baseline_batch(probs, budget_s, sampled):
    """The oracle on sampled block-rows of the batch's problems (two per
    problem, problems in turn) until the budget is spent; the rows it computed
    are then compared with every mode's GPU output of those rows."""
    from oracle import grid as G
    from oracle import operators as O
    info = host_info()
    grids, ops = {}, {}
    t0 = time.perf_counter()
    done = []                     # (problem, J, Cref blocks)
    for i, J in sampled["order"]:
        if done and time.perf_counter() - t0 >= budget_s:
            break
        pr = probs[i]
        lmax = pr["g"].lmax
        if lmax not in grids:
            grids[lmax] = G.make_grid(lmax, 8)
        og = grids[lmax]
        if i not in ops:
            ops[i] = O.LocalOperator(og, pr["b_l"], pr["R"])
        ks = [K for K in og.tile_neighbours(J) if K >= J]
        done.append((i, J, ks, np.stack([O.btnb_block(ops[i], pr["ninv"], J, K) for K in ks])))
    dt = time.perf_counter() - t0
    nblk = sum(len(d[2]) for d in done)
    res = {"value": nblk * 4096 / dt, "unit": "elements/s", "cores": blas_threads(info), "kind": "oracle",
           "sample": f"{len(done)} block-rows ({nblk} stored blocks) drawn two per problem across the 32 "
                     f"problems, grids and unique blocks built on first use inside the {dt:.1f} s wall",
           "host": info}
    gates = {}
    for mode, per in sampled["modes"].items():
        worst, per_prob = 0.0, {}
        for i, J, ks, Cref in done:
            got = per[(i, J)]
            if got["ks"] != ks:
                g_ = float("inf")                      # layout differs from the oracle's neighbours
            else:
                g_ = gate(got["C"], Cref, [J] * len(ks))
            per_prob[i] = max(per_prob.get(i, 0.0), g_)
            worst = max(worst, g_)
        gates[mode] = {"gate": worst, "bound": BOUND[mode], "per_problem": {str(k): v for k, v in per_prob.items()},
                       "rows": len(done)}
    return res, gates


def copy_calibration(torch, nbytes):
    """One plain device copy of nbytes (read and written), launched first so
    that counter runs can scale FETCH_SIZE / WRITE_SIZE by a known size."""
    if nbytes <= 0:
        return
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"# copy calibration: {4 * (nbytes // 4)} bytes read and written", file=sys.stderr, flush=True)
    del src, dst


def run_batch(args):
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    torch.cuda.set_device(0)
    copy_calibration(torch, args.copy_calibration)
    t0 = time.perf_counter()
    probs = batch_inputs(sp, S)
    setup = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    for pr in probs:
        pr["kb"] = sp.Kernel(pr["g"], pr["b_l"], pr["R"], stream=stream)
        pr["ninv_dev"] = torch.as_tensor(pr["ninv"]).cuda()
        pr["out"] = torch.empty(pr["g"].out_len, dtype=torch.float64, device="cuda")
    nelem = sum(pr["g"].nblocks for pr in probs) * 4096
    alg_flop = sum(2.0 * 64 ** 3 * pr["g"].nterms for pr in probs)
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    # sampled rows, two per problem: the first tile and a random one
    rng = np.random.default_rng(11)
    order = []
    for i, pr in enumerate(probs):
        order.append((i, 0))
        order.append((i, int(rng.integers(1, pr["g"].ntiles))))
    order = [order[2 * i] for i in range(32)] + [order[2 * i + 1] for i in range(32)]
    blocks = {}
    for i, pr in enumerate(probs):
        blocks[i] = pr["g"].blocks()
    sampled = {"order": order, "modes": {}}
    print(f"# workload batch32: 32 problems, npix={sum(pr['g'].npix for pr in probs)} "
          f"nblocks={nelem // 4096} output={nelem * 8 / 1e9:.1f} GB setup={setup:.1f}s", file=sys.stderr, flush=True)
    results = {}
    for prec in modes:
        bt = sp.Batch([(pr["g"], pr["kb"], pr["ninv_dev"], pr["out"]) for pr in probs], prec=prec, stream=stream)
        chosen, tune_ms = bt.tune(stream)
        sched = sp.plan_name(chosen)        # "schedule/tiling"
        for _ in range(args.warmup):
            bt.launch(stream)
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t_start = time.perf_counter()
        evs[0].record(stream)
        for i in range(args.steps):
            bt.launch(stream)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        bt.close()
        per = {}
        for i, J in order:
            rp, col = blocks[i]
            n0, n1 = int(rp[J]), int(rp[J + 1])
            per[(i, J)] = {"ks": [int(k) for k in col[n0:n1]],
                           "C": probs[i]["out"].view(-1, 64, 64)[n0:n1].cpu().numpy()}
        sampled["modes"][prec] = per
        ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
        ms_step = wall * 1000.0 / args.steps
        achieved = PRODUCTS[prec] * alg_flop / (ms.mean() * 1e-3) / 1e12
        kern = (BATCH_KERNEL[prec] if chosen % len(sp.SCHEDULES) != sp.SCHED_PER_PROBLEM
                else KERNEL_NAME[prec])
        results[prec] = {
            "elements_per_s": nelem / (ms_step * 1e-3), "ms_per_step": ms_step, "graph_launch_ms": ms.mean(),
            "schedule": sched, "tune_ms": [round(t, 3) for t in tune_ms],
            "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK[prec], "achieved": achieved,
                         "frac": achieved / PEAK[prec], "kernel": kern,
                         "traffic": recorded_traffic(prec, "batch32")},
        }
        print(f"# batch32 batch {prec} ({sched}; tune ms {[round(t, 2) for t in tune_ms]}): step {ms_step:.2f} ms wall, "
              f"{ms.mean():.2f} ms per graph launch, {achieved:.1f} TFLOP/s "
              f"({achieved / PEAK[prec] * 100:.1f}% of {PEAK[prec]} TFLOP/s)", file=sys.stderr, flush=True)
    if "fp64" in results:
        for prec, r in results.items():
            r["speed_vs_fp64"] = r["elements_per_s"] / results["fp64"]["elements_per_s"]
    head = results[modes[0]]
    line = {
        "metric": "B^T N^-1 B elements/s, 32-problem batch in one graph launch",
        "value": head["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[modes[0]],
        "data": "synthetic",
        "config": {"workload": "sympix batch: 32 problems, lmax 256/512/1024/2048 (8 each), "
                               "beam FWHM U[2,5] px cut 3 FWHM, N^-1 U[0.5,2] x cap mask U[0,0.3], "
                               "seeds 5000+p",
                   "problems": 32, "npix": int(sum(pr["g"].npix for pr in probs)),
                   "nblocks": int(nelem // 4096), "precision": modes[0], "schedule": head["schedule"],
                   "tune_ms": head["tune_ms"], "setup_s": round(setup, 2)},
        "roofline": head["roofline"],
        "modes": results,
    }
    if not args.no_cpu_baseline:
        base, gates = cpu_baseline_batch(probs, args.cpu_seconds, sampled)
        line["cpu_baseline"] = base
        for prec, gr in gates.items():
            results[prec]["error_vs_oracle"] = gr
    print(json.dumps(line), flush=True)


def cpu_baseline_conv(cfg, budget_s):
    """The oracle's convolution on random output tiles until the budget is spent."""
    from oracle import grid as G
    from oracle import operators as O
    from workloads import synth as S
    info = host_info()
    threads = blas_threads(info)
    og = G.make_grid(cfg.lmax, cfg.k)
    f = np.random.default_rng(1).standard_normal(og.npix)
    b_l, R = S.gaussian_beam(cfg.lmax, og.npix, cfg.fwhm_pix)
    op = O.LocalOperator(og, b_l, R)
    rng = np.random.default_rng(3)
    t0 = time.perf_counter()
    ntiles = 0
    k2 = og.k ** 2
    refs = {}                            # output tile -> the oracle's g_J, for the comparison
    while time.perf_counter() - t0 < budget_s:
        J = int(rng.integers(og.ntiles))
        acc = np.zeros(k2)
        for K in op.neighbours(J):
            acc += op.block(J, K) @ f[K * k2:(K + 1) * k2]
        refs[J] = acc
        ntiles += 1
    dt = time.perf_counter() - t0
    return {"value": ntiles * k2 / dt, "unit": "pixels/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{ntiles} random output tiles of the lmax={cfg.lmax} convolution, "
                      f"unique blocks evaluated on first use, {dt:.1f} s wall", "host": info}, refs


def run_conv(args):
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    cfg = S.CONFIGS[args.config]
    torch.cuda.set_device(0)
    copy_calibration(torch, args.copy_calibration)
    g = sp.Grid(cfg.lmax, cfg.k)
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    stream = torch.cuda.current_stream()
    kb = sp.Kernel(g, b_l, R, stream=stream)
    f = torch.as_tensor(np.random.default_rng(1).standard_normal(g.npix)).cuda()
    out = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    pairs = g.nadjacency
    alg_flop = 2.0 * 64 * 64 * pairs
    for _ in range(args.warmup):
        sp.convolve(g, kb, f, out, stream=stream)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_start = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        sp.convolve(g, kb, f, out, stream=stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms_step = wall * 1000.0 / args.steps
    achieved = alg_flop / (ms.mean() * 1e-3) / 1e12
    hbm = 16.0 * g.npix / (ms.mean() * 1e-3) / 1e9
    print(f"# conv {args.config}: lmax={cfg.lmax} npix={g.npix} neighbour pairs={pairs}; "
          f"{ms.mean():.3f} ms per call, {achieved:.1f} TFLOP/s ({achieved / PEAK['fp64'] * 100:.1f}% of FP64 "
          f"MFMA peak), f+g {hbm:.0f} GB/s", file=sys.stderr, flush=True)
    line = {
        "metric": "pixel-domain convolution g = B-hat f, output pixels/s",
        "value": g.npix / (ms_step * 1e-3),
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sympix lmax={cfg.lmax} k={cfg.k} beam FWHM {cfg.fwhm_pix:g} px cut 3 FWHM, "
                               f"f ~ N(0,1) seed 1",
                   "lmax": cfg.lmax, "npix": g.npix, "neighbour_pairs": int(pairs)},
        "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK["fp64"], "achieved": achieved,
                     "frac": achieved / PEAK["fp64"], "kernel": "k_convolve",
                     "traffic": recorded_traffic("conv", args.config)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"], refs = cpu_baseline_conv(cfg, args.cpu_seconds)
        # the last timed output on the oracle's tiles (outside the timed region)
        got = out.view(-1, 64).cpu().numpy()
        gate = max(np.abs(got[J] - ref).max() / np.abs(ref).max() for J, ref in refs.items())
        line["error_vs_oracle"] = {"tiles": len(refs), "gate": float(gate), "bound": 1e-10}
        print(f"# conv gate on {len(refs)} tiles: {gate:.2e} (bound 1e-10)", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def cpu_baseline_factor(A, budget_s):
    """The oracle's Cholesky and solve on host copies of sampled diagonal blocks until the budget is spent."""
    from oracle import precond as P
    info = host_info()
    threads = blas_threads(info)
    rng = np.random.default_rng(5)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        U, _ = P.cholesky_upper(A[n % len(A)])
        P.solve_upper_factor(U, rng.standard_normal(A.shape[1]))
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "tiles/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} Cholesky factorisations and solves of 64x64 diagonal blocks A_J = D_JJ + C_JJ "
                      f"({len(A)} random tiles of the workload, copied from the device), {dt:.1f} s wall",
            "host": info}


def run_factor(args):
    """Block-Jacobi preconditioner of D-hat + B-hat^T N^-1 B-hat (Section 4.2): a step is one
    factorisation of every tile's diagonal block and one application to a vector."""
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    cfg = S.CONFIGS[args.config]
    torch.cuda.set_device(0)
    copy_calibration(torch, args.copy_calibration)
    g = sp.Grid(cfg.lmax, cfg.k)
    th, ph = g.pixel_theta_phi()
    ninv = S.ninv_for(cfg, th, ph)
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    stream = torch.cuda.current_stream()
    kb = sp.Kernel(g, b_l, R, stream=stream)
    kd = sp.Kernel(g, S.prior(cfg.lmax), 0.0, stream=stream)
    D = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    C = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    sp.sample_D_BtNB(g, kd, kb, torch.as_tensor(ninv).cuda(), D, C, "fp64", stream=stream)
    U = torch.empty(g.ntiles * 4096, dtype=torch.float64, device="cuda")
    info = torch.empty(g.ntiles, dtype=torch.int32, device="cuda")
    r = torch.as_tensor(np.random.default_rng(2).standard_normal(g.npix)).cuda()
    x = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        sp.factor_diag(g, D, C, U, info, stream=stream)
        sp.solve_diag(g, U, r, x, stream=stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
    t_start = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        sp.factor_diag(g, D, C, U, info, stream=stream)
        ev[2 * i + 1].record(stream)
        sp.solve_diag(g, U, r, x, stream=stream)
        ev[2 * i + 2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    f_ms = np.array([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps)])
    s_ms = np.array([ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(args.steps)])
    ms_step = wall * 1000.0 / args.steps
    f_bytes = g.ntiles * (3 * 4096 * 8 + 4)            # D_JJ and C_JJ read, U_J written, info
    s_bytes = g.ntiles * 4096 * 8 + 2 * 8 * g.npix      # U read, r read, x written
    f_gbs = f_bytes / (f_ms.mean() * 1e-3) / 1e9
    s_gbs = s_bytes / (s_ms.mean() * 1e-3) / 1e9
    info_h = info.cpu().numpy()
    tiles_b, _, _ = g.bands()
    band_of = np.repeat(np.arange(len(tiles_b)), tiles_b)
    failed_bands = sorted(set(band_of[info_h > 0].tolist()))
    print(f"# factor {args.config}: lmax={cfg.lmax} tiles={g.ntiles}; factor {f_ms.mean():.3f} ms "
          f"({f_gbs:.0f} GB/s), solve {s_ms.mean():.3f} ms ({s_gbs:.0f} GB/s); step {ms_step:.3f} ms; "
          f"failed pivots {int((info_h > 0).sum())} in bands {failed_bands[:10]}", file=sys.stderr, flush=True)
    line = {
        "metric": "block-Jacobi factor and solve of D-hat + B-hat^T N^-1 B-hat, tiles/s",
        "value": g.ntiles / (ms_step * 1e-3),
        "unit": "tiles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sympix lmax={cfg.lmax} k={cfg.k}: FP64 D-hat (prior (l+1)^2) and B-hat^T N^-1 "
                               f"B-hat (beam FWHM {cfg.fwhm_pix:g} px, N^-1 {cfg.ninv_kind} seed {cfg.seed}) "
                               f"diagonal blocks; r ~ N(0,1) seed 2",
                   "lmax": cfg.lmax, "ntiles": g.ntiles, "npix": g.npix},
        "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK, "achieved": f_gbs,
                     "frac": f_gbs / HBM_PEAK, "kernel": "k_factor_diag",
                     "traffic": recorded_traffic("factor", args.config, "precond.hip")},
        "factor_ms": float(f_ms.mean()),
        "solve": {"ms": float(s_ms.mean()), "kernel": "k_solve_diag", "achieved_GBs": s_gbs,
                  "frac": s_gbs / HBM_PEAK, "traffic": recorded_traffic("solve", args.config, "precond.hip")},
        "failed_pivots": int((info_h > 0).sum()),
        "failed_bands": failed_bands,
    }
    if not args.no_cpu_baseline:
        brp, _ = g.blocks()
        pick = np.random.default_rng(4).choice(g.ntiles, 256, replace=False)
        pick = pick[info_h[pick] == 0]
        idx = torch.as_tensor(brp[pick], device="cuda")
        A = (D.view(-1, 64, 64)[idx] + C.view(-1, 64, 64)[idx]).cpu().numpy()
        line["cpu_baseline"] = cpu_baseline_factor(A, args.cpu_seconds)
        # the last timed outputs of the same tiles against the oracle (outside the timed region):
        # the GPU factor's backward error, and both factors and solves relative to kappa(A_J)
        from oracle import precond as P
        Ug = U.view(-1, 64, 64)[torch.as_tensor(pick, device="cuda")].cpu().numpy()
        xg = x.view(-1, 64)[torch.as_tensor(pick, device="cuda")].cpu().numpy()
        rh = r.view(-1, 64)[torch.as_tensor(pick, device="cuda")].cpu().numpy()
        back = fwd = sol = 0.0
        for n in range(len(pick)):
            a = np.triu(A[n]) + np.triu(A[n], 1).T
            ev = np.linalg.eigvalsh(a)
            kappa = ev[-1] / ev[0]
            Uo, _ = P.cholesky_upper(A[n])
            back = max(back, np.abs(Ug[n].T @ Ug[n] - a).max() / np.abs(a).max())
            fwd = max(fwd, np.abs(Ug[n] - Uo).max() / np.abs(Uo).max() / kappa)
            xo = P.solve_upper_factor(Uo, rh[n])
            sol = max(sol, np.abs(xg[n] - xo).max() / np.abs(xo).max() / kappa)
        line["error_vs_oracle"] = {"tiles": int(len(pick)), "factor_backward": back, "factor_forward_over_kappa": fwd,
                                   "solve_over_kappa": sol, "bound_backward": 4 * 64 * 2.0 ** -52}
        print(f"# factor gate on {len(pick)} tiles: backward {back:.2e} (bound {4 * 64 * 2.0 ** -52:.1e}), "
              f"factor/kappa {fwd:.2e}, solve/kappa {sol:.2e}", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def sht_terms(nrings, L):
    """(degree, order, ring) triples of one Legendre pass: nrings (L+1)(L+2)/2."""
    return nrings * (L + 1) * (L + 2) // 2


def cpu_baseline_sht(budget_s):
    """The oracle's synthesis and analysis (whole grid, lmax 256, L = 256) until the budget is spent."""
    from oracle import grid as G
    from oracle import sht as H
    info = host_info()
    threads = blas_threads(info)
    L = 256
    og = G.make_grid(L, 8)
    a = np.random.default_rng(4).standard_normal((L + 1) ** 2)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        H.analysis(og, H.synthesis(og, a, L), L)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n * 2 * sht_terms(og.nrings, L) / dt, "unit": "Legendre terms/s", "cores": int(threads),
            "kind": "oracle", "sample": f"{n} synthesis + analysis round trips at lmax 256 (whole grid, L = 256), "
                                       f"{dt:.1f} s wall", "host": info}


def run_sht(args):
    """Spherical harmonic synthesis + analysis (one round trip per step) at L =
    lmax on the grid, and the degrade of Eq. 14 onto a grid of half the band
    limit (timed apart)."""
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    cfg = S.CONFIGS[args.config]
    torch.cuda.set_device(0)
    copy_calibration(torch, args.copy_calibration)
    L = cfg.lmax
    g = sp.Grid(cfg.lmax, cfg.k)
    s = sp.Sht(g, L)
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(cfg.seed + 21)
    ell = np.repeat(np.arange(L + 1), 2 * np.arange(L + 1) + 1)
    a = torch.as_tensor(rng.standard_normal((L + 1) ** 2) / np.sqrt(ell + 1.0)).cuda()
    f = torch.empty(g.npix, dtype=torch.float64, device="cuda")
    back = torch.empty_like(a)
    for _ in range(args.warmup):
        s.synthesis(a, f, stream=stream)
        s.analysis(f, back, stream=stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        s.synthesis(a, f, stream=stream)
        ev[i][1].record(stream)
        s.analysis(f, back, stream=stream)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    t_syn = np.array([e[0].elapsed_time(e[1]) for e in ev])
    t_ana = np.array([e[1].elapsed_time(e[2]) for e in ev])
    ms_step = wall * 1000.0 / args.steps
    rt_err = float((back - a).abs().max() / a.abs().max())
    # degrade onto a grid of half the band limit (L_2 = lmax / 2 on both plans)
    L2 = cfg.lmax // 2
    g2 = sp.Grid(L2, cfg.k)
    so, s2 = sp.Sht(g, L2), sp.Sht(g2, L2)
    th = torch.as_tensor(S.ninv_for(cfg, *g.pixel_theta_phi())).cuda()
    th2 = torch.empty(g2.npix, dtype=torch.float64, device="cuda")
    sp.degrade(so, s2, th, th2, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        sp.degrade(so, s2, th, th2, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_deg = e0.elapsed_time(e1) / 3
    terms = sht_terms(g.nrings, L)
    # one Legendre pass: per (degree, order, ring pair) a recurrence step (a
    # multiply and a fused multiply-add) and two fused multiply-adds, 7 flops
    flop = 7.0 * (g.nrings // 2) * (L + 1) * (L + 2) / 2
    achieved = flop / (t_syn.mean() * 1e-3) / 1e12
    print(f"# sht {args.config}: lmax={cfg.lmax} L={L} npix={g.npix} nrings={g.nrings}; synthesis "
          f"{t_syn.mean():.3f} ms, analysis {t_ana.mean():.3f} ms, round trip error {rt_err:.1e}; degrade "
          f"lmax {cfg.lmax} -> {L2} (L={L2}) {t_deg:.3f} ms; Legendre part {achieved:.1f} TFLOP/s "
          f"({achieved / FP64_VECTOR * 100:.1f}% of FP64 vector peak, whole synthesis call)",
          file=sys.stderr, flush=True)
    line = {
        "metric": "spherical harmonic synthesis + analysis, Legendre terms/s",
        "value": 2 * terms / (ms_step * 1e-3),
        "unit": "Legendre terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sympix lmax={cfg.lmax} k={cfg.k}, L={L}, a_lm ~ N(0, 1/(l+1)) seed "
                               f"{cfg.seed + 21}; degrade of the N^-1 map onto lmax {L2}",
                   "lmax": cfg.lmax, "L": L, "npix": g.npix, "nrings": g.nrings},
        "modes": {"synthesis_ms": float(t_syn.mean()), "analysis_ms": float(t_ana.mean()),
                  "degrade_ms": float(t_deg), "round_trip_error": rt_err},
        "roofline": {"bound": "alu", "unit": "TFLOP/s", "peak": FP64_VECTOR, "achieved": achieved,
                     "frac": achieved / FP64_VECTOR, "kernel": "k_leg_syn (whole synthesis call timed)",
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_sht(args.cpu_seconds)
        # the last timed synthesis on the equator ring against the oracle's sums there
        # (outside the timed region; the oracle takes about 25 s for one ring at L = 3000)
        from oracle import grid as G
        from oracle import sht as H
        og = G.make_grid(cfg.lmax, cfg.k)
        r_eq = og.nrings // 2
        ring_of, _, _, _ = og.pixel_coords()
        t0 = time.perf_counter()
        f_ref = H.synthesis(og, a.cpu().numpy(), L, rings=[r_eq])
        dt = time.perf_counter() - t0
        f_got = f.cpu().numpy()[ring_of == r_eq]
        gr = float(np.abs(f_got - f_ref).max() / np.abs(f_ref).max())
        line["error_vs_oracle"] = {"ring": int(r_eq), "pixels": int(f_ref.size), "synthesis_gate": gr,
                                   "oracle_s": dt}
        print(f"# sht gate on ring {r_eq} ({f_ref.size} pixels): {gr:.2e}, oracle {dt:.0f} s", file=sys.stderr,
              flush=True)
    print(json.dumps(line), flush=True)


def cpu_baseline_two_hop(cfg, ninv, b_l, R, rp, col, budget_s):
    """The oracle's B^T N^-1 B blocks of random two-hop block-rows until the budget is spent; returns
    the baseline and, per block computed, its position in the pattern and the oracle's values."""
    from oracle import grid as G
    from oracle import operators as O
    info = host_info()
    threads = blas_threads(info)
    og = G.make_grid(cfg.lmax, cfg.k)
    op = O.LocalOperator(og, b_l, R)
    rng = np.random.default_rng(cfg.seed + 13)
    idx, rows, refs = [], [], []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        J = int(rng.integers(og.ntiles))
        for n in range(int(rp[J]), int(rp[J + 1])):
            refs.append(O.btnb_block(op, ninv, J, int(col[n])))
            idx.append(n)
            rows.append(J)
    dt = time.perf_counter() - t0
    return ({"value": len(idx) * 4096 / dt, "unit": "elements/s", "cores": int(threads), "kind": "oracle",
             "sample": f"{len(set(rows))} random block-rows ({len(idx)} blocks) of the lmax={cfg.lmax} two-hop "
                       f"pattern, unique blocks evaluated on first use, {dt:.1f} s wall", "host": info},
            idx, rows, np.stack(refs) if refs else np.zeros((0, 64, 64)))


def run_two_hop(args):
    """B^T N^-1 B on the two-hop pattern (every nonzero block of the product)."""
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    cfg = S.CONFIGS[args.config]
    prec = [m.strip() for m in args.modes.split(",") if m.strip()][0]
    torch.cuda.set_device(0)
    g = sp.Grid(cfg.lmax, cfg.k)
    t0 = time.perf_counter()
    nblk, nterms = g.pattern_size("two_hop")
    setup = time.perf_counter() - t0
    th, ph = g.pixel_theta_phi()
    ninv = S.ninv_for(cfg, th, ph)
    ninv_dev = torch.as_tensor(ninv).cuda()
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    out = torch.empty(nblk * 4096, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    nelem = nblk * 4096
    alg_flop = 2.0 * 64 ** 3 * nterms
    print(f"# two-hop {args.config} {prec}: lmax={cfg.lmax} blocks={nblk} (one-hop {g.nblocks}) terms={nterms} "
          f"output={nelem * 8 / 1e9:.1f} GB pattern_setup={setup:.2f}s", file=sys.stderr, flush=True)

    def step(ev):
        ev[0].record(stream)
        kb = sp.Kernel(g, b_l, R, stream=stream)
        ev[1].record(stream)
        sp.sample_BtNB_pattern(g, kb, ninv_dev, out, prec, "two_hop", stream=stream)
        ev[2].record(stream)
        return kb

    for _ in range(args.warmup):
        keep = step([torch.cuda.Event(enable_timing=True) for _ in range(3)])
        torch.cuda.synchronize()
        del keep
    evs, keeps = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        keeps.append(step(ev))
        evs.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    keeps.clear()
    t_C = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_step = wall * 1000.0 / args.steps
    mfma = PRODUCTS[prec] * alg_flop / (t_C * 1e-3) / 1e12
    gbs = nelem * 8 / (t_C * 1e-3) / 1e9
    t_mfma = PRODUCTS[prec] * alg_flop / (PEAK[prec] * 1e12)
    t_hbm = nelem * 8 / (HBM_PEAK * 1e9)
    if t_hbm >= t_mfma:
        roof = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK, "achieved": gbs, "frac": gbs / HBM_PEAK,
                "mfma_frac": mfma / PEAK[prec]}
    else:
        roof = {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK[prec], "achieved": mfma, "frac": mfma / PEAK[prec],
                "hbm_frac": gbs / HBM_PEAK}
    roof["kernel"] = KERNEL_NAME[prec]
    roof["traffic"] = None
    print(f"# two-hop {prec}: step {ms_step:.2f} ms, contraction {t_C:.2f} ms, {mfma:.1f} TFLOP/s "
          f"({mfma / PEAK[prec] * 100:.1f}% of {PEAK[prec]} TFLOP/s), {gbs:.0f} GB/s written",
          file=sys.stderr, flush=True)
    line = {
        "metric": "B^T N^-1 B elements/s, two-hop pattern (every nonzero block of the product)",
        "value": nelem / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": f"sympix lmax={cfg.lmax} k={cfg.k} two-hop blocks, beam FWHM {cfg.fwhm_pix:g} px "
                               f"cut 3 FWHM, N^-1 {cfg.ninv_kind} seed {cfg.seed}",
                   "lmax": cfg.lmax, "nblocks": nblk, "nterms": nterms, "precision": prec},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        rp, col = g.pattern_blocks("two_hop")
        base, idx, rows, ref = cpu_baseline_two_hop(cfg, ninv, b_l, R, rp, col, args.cpu_seconds)
        line["cpu_baseline"] = base
        # the last timed output on the oracle's blocks (outside the timed region)
        got = out.view(-1, 64, 64)[torch.as_tensor(np.asarray(idx, dtype=np.int64), device="cuda")].cpu().numpy()
        gr = gate(got, ref, rows)
        line["error_vs_oracle"] = {"blocks": len(idx), "gate": gr, "bound": BOUND[prec]}
        print(f"# two-hop gate on {len(idx)} blocks: {gr:.2e} (bound {BOUND[prec]:g})", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def cpu_baseline_two_grid(cfg, lmax2, ninv2, b_l, R, rp, col, budget_s):
    """The oracle's B^T N_2^-1 B blocks of random block-rows of Y_1 until the budget is spent; returns
    the baseline and, per block computed, its position in the stored-block order and its values."""
    from oracle import grid as G
    from oracle import twogrid as X
    info = host_info()
    threads = blas_threads(info)
    og1, og2 = G.make_grid(cfg.lmax, cfg.k), G.make_grid(lmax2, cfg.k)
    op = X.CrossOperator(og2, og1, b_l, R)
    rng = np.random.default_rng(cfg.seed + 17)
    idx, rows, refs = [], [], []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        J = int(rng.integers(og1.ntiles))
        for n in range(int(rp[J]), int(rp[J + 1])):
            refs.append(X.btnb_cross_block(op, ninv2, J, int(col[n])))
            idx.append(n)
            rows.append(J)
    dt = time.perf_counter() - t0
    return ({"value": len(idx) * 4096 / dt, "unit": "elements/s", "cores": int(threads), "kind": "oracle",
             "sample": f"{len(set(rows))} random block-rows ({len(idx)} blocks) of Y_1 (lmax {cfg.lmax}) with "
                       f"N_2^-1 on Y_2 (lmax {lmax2}), unique blocks evaluated on first use, {dt:.1f} s wall",
             "host": info},
            idx, rows, np.stack(refs) if refs else np.zeros((0, 64, 64)))


def run_two_grid(args):
    """B^T N_2^-1 B with N_2^-1 on an auxiliary grid Y_2 of twice the band limit
    (Eq. 13; Section 4.2's "twice that of Y_1"): a step tabulates the two-grid
    beam kernel and contracts, in the first of --modes."""
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    cfg = S.CONFIGS[args.config]
    lmax2 = args.lmax2 or 2 * cfg.lmax
    prec = [m.strip() for m in args.modes.split(",") if m.strip()][0]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g1, g2 = sp.Grid(cfg.lmax, cfg.k), sp.Grid(lmax2, cfg.k)
    x = sp.Cross(g2, g1)
    setup = time.perf_counter() - t0
    th2, ph2 = g2.pixel_theta_phi()
    ninv2_h = S.ninv_for(cfg, th2, ph2)
    ninv2 = torch.as_tensor(ninv2_h).cuda()
    b_l, R = S.gaussian_beam(cfg.lmax, g1.npix, cfg.fwhm_pix)
    out = torch.empty(x.out_len, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    nelem = x.nblocks * 4096
    alg_flop = 2.0 * 64 ** 3 * x.nterms
    print(f"# two-grid {args.config}: lmax1={cfg.lmax} lmax2={lmax2} npix2={g2.npix} blocks={x.nblocks} "
          f"terms={x.nterms} (max {x.max_terms}) unique={x.nunique} setup={setup:.2f}s", file=sys.stderr, flush=True)

    def step(ev):
        ev[0].record(stream)
        kb = sp.CrossKernel(x, b_l, R, stream=stream)
        ev[1].record(stream)
        sp.sample_BtNB_cross(x, kb, ninv2, out, prec, stream=stream)
        ev[2].record(stream)
        return kb

    for _ in range(args.warmup):
        keep = step([torch.cuda.Event(enable_timing=True) for _ in range(3)])
        torch.cuda.synchronize()
        del keep
    evs, keeps = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        keeps.append(step(ev))
        evs.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    keeps.clear()
    t_C = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    t_T = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    ms_step = wall * 1000.0 / args.steps
    mfma = PRODUCTS[prec] * alg_flop / (t_C * 1e-3) / 1e12
    print(f"# two-grid {prec}: step {ms_step:.2f} ms, contraction {t_C:.2f} ms ({mfma:.1f} TFLOP/s, "
          f"{mfma / PEAK[prec] * 100:.1f}% of {PEAK[prec]}), tabulation {t_T:.2f} ms", file=sys.stderr, flush=True)
    line = {
        "metric": "B^T N_2^-1 B elements/s, N_2^-1 on an auxiliary grid of twice the band limit",
        "value": nelem / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": f"sympix Y_1 lmax={cfg.lmax}, Y_2 lmax={lmax2}, k={cfg.k}, beam FWHM "
                               f"{cfg.fwhm_pix:g} px of Y_1 cut 3 FWHM, N_2^-1 {cfg.ninv_kind} seed {cfg.seed} on Y_2",
                   "lmax1": cfg.lmax, "lmax2": lmax2, "nblocks": x.nblocks, "nterms": x.nterms, "precision": prec,
                   "tabulate_ms": t_T, "contraction_ms": t_C},
        "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK[prec], "achieved": mfma,
                     "frac": mfma / PEAK[prec], "kernel": KERNEL_NAME[prec], "traffic": None},
    }
    if not args.no_cpu_baseline:
        rp, col = g1.blocks()
        base, idx, rows, ref = cpu_baseline_two_grid(cfg, lmax2, ninv2_h, b_l, R, rp, col, args.cpu_seconds)
        line["cpu_baseline"] = base
        # the last timed output on the oracle's blocks (outside the timed region)
        got = out.view(-1, 64, 64)[torch.as_tensor(np.asarray(idx, dtype=np.int64), device="cuda")].cpu().numpy()
        gr = gate(got, ref, rows)
        line["error_vs_oracle"] = {"blocks": len(idx), "gate": gr, "bound": BOUND[prec]}
        print(f"# two-grid gate on {len(idx)} blocks: {gr:.2e} (bound {BOUND[prec]:g})", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the sampling path runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding the grid by band pairs across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.config == "batch32":
        run_batch(args)
        return
    if args.op == "conv":
        run_conv(args)
        return
    if args.op == "two_hop":
        run_two_hop(args)
        return
    if args.op == "two_grid":
        run_two_grid(args)
        return
    if args.op == "sht":
        run_sht(args)
        return
    if args.op == "factor":
        run_factor(args)
        return
    import torch

    import paper_1504_04653_amd as sp
    from workloads import synth as S

    cfg = S.CONFIGS[args.config]
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    torch.cuda.set_device(0)

    t0 = time.perf_counter()
    g = sp.Grid(cfg.lmax, cfg.k)
    setup_grid = time.perf_counter() - t0
    th, ph = g.pixel_theta_phi()
    ninv = S.ninv_for(cfg, th, ph)
    b_l, R = S.gaussian_beam(cfg.lmax, g.npix, cfg.fwhm_pix)
    d_l = S.prior(cfg.lmax)
    ninv_dev = torch.as_tensor(ninv).cuda()
    out_C = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    out_D = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    nelem = g.nblocks * 4096
    alg_flop = 2.0 * 64 ** 3 * g.nterms
    print(f"# workload {args.config}: lmax={cfg.lmax} npix={g.npix} nblocks={g.nblocks} "
          f"nterms={g.nterms} nunique={g.nunique} grid_setup={setup_grid:.2f}s", file=sys.stderr, flush=True)
    # block-rows whose outputs are kept for the comparison with the oracle
    blk_ptr, blk_col = g.blocks()
    rows = sampled_rows(g.bands()[0], 160, seed=cfg.seed + 7)
    sidx, spairs = row_blocks(blk_ptr, blk_col, rows)
    sidx_t = torch.as_tensor(sidx, device="cuda")
    sampled = {"rows": rows, "pairs": spairs, "modes": {}}

    copy_calibration(torch, args.copy_calibration)

    def roofline(prec, t_ms, fused):
        """The binding roof of the contraction launch: MFMA work at the dense
        peak of its operand type, or (when the launch also writes D-hat) HBM
        writes at 8 TB/s, whichever takes longer; the other is kept beside."""
        mfma = PRODUCTS[prec] * alg_flop / (t_ms * 1e-3) / 1e12
        r_mfma = {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK[prec], "achieved": mfma,
                  "frac": mfma / PEAK[prec]}
        if not fused:
            return r_mfma
        written = 2 * nelem * 8                      # B^T N^-1 B and D-hat, FP64
        t_mfma = PRODUCTS[prec] * alg_flop / (PEAK[prec] * 1e12)
        t_hbm = written / (HBM_PEAK * 1e9)
        gbs = written / (t_ms * 1e-3) / 1e9
        r_hbm = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK, "achieved": gbs, "frac": gbs / HBM_PEAK}
        if t_hbm >= t_mfma:
            r_hbm["mfma_frac"] = r_mfma["frac"]
            return r_hbm
        r_mfma["hbm_frac"] = r_hbm["frac"]
        return r_mfma

    fused = not args.separate

    # One step: tabulate the beam and prior kernels (with their unique
    # blocks), then sample D-hat and B^T N^-1 B.  Events: 0 start, 1 kernels
    # tabulated, 2 D-hat done (separate calls) or both done (combined call),
    # 3 step done.
    def step(prec, ev):
        ev[0].record(stream)
        kb = sp.Kernel(g, b_l, R, stream=stream)
        kd = sp.Kernel(g, d_l, 0.0, stream=stream)
        ev[1].record(stream)
        sample(prec, kb, kd, ev, first=False)
        return kb, kd

    # Pipelined steps (default): the kernels of step s + 1 are tabulated on a
    # second stream (default priority) while step s samples on the main
    # stream; the main stream waits for them before sampling.  Every step still
    # tabulates both kernels and writes both outputs.
    tab_stream = torch.cuda.Stream()

    def tabulate(st):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        kb = sp.Kernel(g, b_l, R, stream=st)
        kd = sp.Kernel(g, d_l, 0.0, stream=st)
        ev1.record(st)
        return kb, kd, ev0, ev1

    def sample(prec, kb, kd, ev, first=True):
        if first:
            ev[1].record(stream)
        if not fused:
            sp.sample_D(g, kd, out_D, stream=stream)
            ev[2].record(stream)
            sp.sample_BtNB(g, kb, ninv_dev, out_C, prec, stream=stream)
        else:
            sp.sample_D_BtNB(g, kd, kb, ninv_dev, out_D, out_C, prec, stream=stream)
            ev[2].record(stream)
        ev[3].record(stream)

    def run_overlapped(prec, nsteps):
        evs, keeps = [], []
        nxt = tabulate(tab_stream)
        for s_ in range(nsteps):
            kb, kd, t0, t1 = nxt
            stream.wait_event(t1)
            ev = [t0] + [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            if s_ + 1 < nsteps:                 # queued behind this step's tabulation on its stream
                nxt = tabulate(tab_stream)
            sample(prec, kb, kd, ev)
            keeps.append((kb, kd))
            evs.append((ev, t1))
        return evs, keeps

    def contraction_alone(prec, kb, n=3):
        """Untimed comparison: the contraction alone in the class-kernel grid
        (sample_BtNB) and as a one-problem persistent batch in one captured
        graph (tuned over its schedules and tile shapes)."""
        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
            e[0].record(stream)
            for i in range(n):
                fn()
                e[i + 1].record(stream)
            torch.cuda.synchronize()
            return float(np.mean([e[i].elapsed_time(e[i + 1]) for i in range(n)]))
        t_grid = timed(lambda: sp.sample_BtNB(g, kb, ninv_dev, out_C, prec, stream=stream))
        bt = sp.Batch([(g, kb, ninv_dev, out_C)], prec=prec, stream=stream)
        chosen, _ = bt.tune(stream)
        t_batch = timed(lambda: bt.launch(stream))
        bt.close()
        return {"class_grid_ms": t_grid, "persistent_batch_ms": t_batch, "batch_plan": sp.plan_name(chosen),
                "class_grid_kernel": KERNEL_NAME[prec], "batch_kernel": BATCH_KERNEL[prec]}

    results = {}
    for prec in modes:
        if args.no_overlap:
            for _ in range(args.warmup):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                keep = step(prec, ev)
                torch.cuda.synchronize()
                del keep
        else:
            run_overlapped(prec, max(1, args.warmup))
        evs = []
        keeps = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        if args.no_overlap:
            for _ in range(args.steps):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                keeps.append(step(prec, ev))   # kernel handles are freed after the final synchronisation
                evs.append(ev)
        else:
            evo, keeps = run_overlapped(prec, args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        # the sampled rows of this mode's last timed outputs, for the oracle comparison
        sampled["modes"][prec] = {"C": out_C.view(-1, 64, 64)[sidx_t].cpu().numpy(),
                                  "D": out_D.view(-1, 64, 64)[sidx_t].cpu().numpy() if fused else None}
        kb_last = keeps[-1][0]
        if args.no_overlap:
            seg = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                             e[0].elapsed_time(e[3])] for e in evs])   # ms
        else:   # tabulation: its own stream's events; the step: sampling (the tabulation overlaps)
            seg = np.array([[e[0].elapsed_time(t1), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                             e[1].elapsed_time(e[3])] for e, t1 in evo])
        t_tab, t_a, t_b, t_step = seg.mean(axis=0)
        # separate calls: t_a = D-hat, t_b = contraction; combined call: t_a =
        # both outputs (one launch)
        t_D, t_C = (None, t_a) if fused else (t_a, t_b)
        ms_step = wall * 1000.0 / args.steps
        r = {
            "elements_per_s": nelem / (ms_step * 1e-3),
            "ms_per_step": ms_step,
            "step_events_ms": t_step,
            "tabulate_ms": t_tab,
            "tabulation_overlapped": not args.no_overlap,
            "D_and_btnb_one_launch": fused,
            "btnb_ms": t_C,
            "btnb_elements_per_s": nelem / (t_C * 1e-3),
            "btnb_tflops_algorithmic": alg_flop / (t_C * 1e-3) / 1e12,
            "btnb_roofline": roofline(prec, t_C, fused),
        }
        if fused:       # the launch also writes the D-hat blocks
            r["hbm_write_GBs"] = 2 * nelem * 8 / (t_C * 1e-3) / 1e9
        else:
            r["D_ms"] = t_D
            r["D_hbm_GBs"] = nelem * 8 / (t_D * 1e-3) / 1e9
        if not args.no_batch_compare:
            r["contraction_alone"] = contraction_alone(prec, kb_last)
        keeps.clear()
        del kb_last
        results[prec] = r
        dpart = (f"D-hat in the same launch ({r['hbm_write_GBs']:.0f} GB/s written)" if fused
                 else f"D {t_D:.2f} ms ({r['D_hbm_GBs']:.0f} GB/s)")
        rf = r["btnb_roofline"]
        ca = r.get("contraction_alone")
        cpart = (f"; contraction alone {ca['class_grid_ms']:.2f} ms in the class grid, "
                 f"{ca['persistent_batch_ms']:.2f} ms as a persistent batch ({ca['batch_plan']})" if ca else "")
        print(f"# {prec}: step {ms_step:.2f} ms, btnb {t_C:.2f} ms "
              f"({rf['frac'] * 100:.1f}% of {rf['peak']} {rf['unit']}"
              f"{', MFMA %.1f%%' % (rf['mfma_frac'] * 100) if 'mfma_frac' in rf else ''}), {dpart}, "
              f"tabulate {t_tab:.2f} ms, step by events {t_step:.2f} ms{cpart}",
              file=sys.stderr, flush=True)

    head = HEADLINE if HEADLINE in results else modes[0]
    hr = results[head]
    if "fp64" in results:
        for prec, r in results.items():
            r["speed_vs_fp64"] = r["elements_per_s"] / results["fp64"]["elements_per_s"]
    # the committed counter rows are taken on the default step (combined call)
    traffic = recorded_traffic(head, args.config) if fused else None
    roof = dict(hr["btnb_roofline"])
    roof["kernel"] = KERNEL_NAME[head]
    if hr["D_and_btnb_one_launch"]:
        roof["kernel"] = roof["kernel"].replace("false", "true")   # the instantiation that also writes D-hat
        roof["note"] = (f"one launch writes B^T N^-1 B and D-hat ({2 * nelem * 8 / 1e9:.1f} GB); its lower bound "
                        "is the larger of the MFMA time and the HBM write time")
    roof["traffic"] = traffic
    line = {
        "metric": METRIC,
        "value": hr["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"sympix lmax={cfg.lmax} k={cfg.k} beam FWHM {cfg.fwhm_pix:g} px "
                               f"cut 3 FWHM, prior (l+1)^2, N^-1 {cfg.ninv_kind} seed {cfg.seed}",
                   "lmax": cfg.lmax, "k": cfg.k, "npix": g.npix, "nblocks": g.nblocks,
                   "nterms": g.nterms, "nunique": g.nunique, "precision": head,
                   "grid_setup_s": round(setup_grid, 3)},
        "roofline": roof,
        "modes": results,
    }
    if not args.no_cpu_baseline:
        base, gates = cpu_baseline(cfg, g, args.cpu_seconds, args.cpu_seconds_1t, sampled)
        line["cpu_baseline"] = base
        line["gates"] = {m: gr["C"]["gate"] for m, gr in gates.items()}
        for prec, gr in gates.items():
            results[prec]["error_vs_oracle"] = gr
        print("# gates against the oracle: " + ", ".join(
            f"{m} {gr['C']['gate']:.2e} (bound {gr['bound']:.0e})" + (f", D {gr['D']['gate']:.2e}" if "D" in gr else "")
            for m, gr in gates.items()), file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
