#!/usr/bin/env python3
"""Benchmark: 512^3 survey-like reconstructions per second on one MI355X.

One step is one whole reconstruction of the survey-like workload: deposit of
galaxies and randoms, totals / smoothing / mask / overdensity / starting
displacement, correction passes until eps <= tol, and the shift of galaxies
and randoms.  Inputs are generated on the host, copied to HBM once, and are
resident before the timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
START_NAMES = {"plain": 0, "ffta1": 1, "ffta2": 2, "learned": 3}
RELAXED_SUFFIX = "_relaxed"   # a start name with this suffix runs the relaxed correction pass (RECON_RELAXED)


def start_of(name):
    """(start code, relaxed) of a start name such as 'learned' or 'plain_relaxed'."""
    relaxed = name.endswith(RELAXED_SUFFIX)
    return START_NAMES[name[:-len(RELAXED_SUFFIX)] if relaxed else name], relaxed


BRICK = 16
BIN_BLOCKS = 256          # binning blocks (recon_tuning.h RECON_BIN_BLOCKS), 16384 objects each at least


def bin_blocks(count):
    return min(BIN_BLOCKS, (count + 16383) // 16384)


def touched_bricks(pos, n, box_len):
    """16^3 bricks the brick-binned deposit of these objects touches: those holding an object's base cell
    and their upper neighbours (a brick's stencil footprint reaches one cell into them).  The integer
    grids are brick-sparse, so these are the bricks that are cleared, written and read back."""
    import numpy as np
    nbs = n // BRICK
    cell = np.floor(pos.astype(np.float64) * (n / box_len)).astype(np.int64) % n
    b = cell // BRICK
    occ = np.zeros((nbs, nbs, nbs), dtype=bool)
    occ[b[:, 2], b[:, 1], b[:, 0]] = True
    out = np.zeros_like(occ)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                out |= np.roll(occ, (dz, dy, dx), axis=(0, 1, 2))
    return int(out.sum())


def algorithmic_bytes(n, n_gal, n_ran, randoms=True, keep_delta=False, bricks_g=None, bricks_r=None, levels=1,
                      tiles=None):
    """Compulsory bytes of one launch of each kernel kind (inputs read once, outputs written once).

    cn = (N/2+1) N^2 complex spectrum elements (8 B), n3 = N^3 cells.  The int64 deposit grids are
    brick-sparse: only the touched bricks (bricks_g, bricks_r; all when None) are written and read.
    tiles = (galaxy-grid tiles with data, random-grid tiles with data, tiles inside the mask, tiles) of
    the setup transforms (recon_tile_counts; all tiles when None): the forward z pass writes, and the
    forward y pass reads, only the grid tiles with data; the inverse y pass writes, the overdensity
    step reads and writes, and the y pass of D_s reads only the tiles inside the mask.
    """
    n3 = n ** 3
    cn = (n // 2 + 1) * n * n * 8
    na = 2 if randoms else 1
    nbs3 = (n // BRICK) ** 3
    gb = (nbs3 if bricks_g is None else bricks_g) * BRICK ** 3 * 8      # galaxy grid bytes held
    rb = (nbs3 if bricks_r is None else bricks_r) * BRICK ** 3 * 8 if randoms else 0
    if tiles is None:
        fg, fr, fm = 1.0, (1.0 if randoms else 0.0), 1.0
    else:
        fg, fr, fm = tiles[0] / tiles[3], tiles[1] / tiles[3], tiles[2] / tiles[3]
    return {
        "z_iter": 4 * cn,                       # 2 spectra in (combined state), 2 out
        "y_fanout": 4 * cn,                     # 2 in, 2 out (combined); the output's full form: 2 in, 3 out
        "y_fanin": 4 * cn,                      # 2 in, 2 out
        "x_iter": 7 * cn,                       # A, B, D_s, D_n in; D_n+1, 2 spectra out
        "z_final": 3 * cn + 3 * n3 * 4,         # 3 spectra in, Psi (3 real fields) out
        "y_fanout_full": 5 * cn,
        "z_final_u": 2 * cn + n3 * 4,           # combined state in, u out (learned start)
        "z_fwd_grid": gb + rb + (fg + fr) * cn,  # touched bricks of the int64 grids in, their tiles' spectra out
        "x_smooth": na * 2 * cn,
        # inside the mask's tiles: the smoothed spectra and the mask in, the overdensity's spectrum out; the
        # kept delta_s is written whole
        "z_delta": (fm * (2 * cn + n3 + cn) if randoms else 2 * cn) + (n3 * 4 if keep_delta else 0),
        "x_start": cn + 3 * cn,
        "totals": na * n3 * 8,
        # touched bricks of the random grid in, 1 B per cell out; the mask read again for its tile flags
        "mask": rb + 2 * n3 if randoms else 0,
        "paint_grids": gb + rb,                 # touched bricks cleared and written (both catalogues)
        "paint": None,                          # per catalogue: 12 B per object + grid written once
        # per catalogue: 24 B per object (position in, displacement out) + the three Psi components at the
        # nodes the objects' stencils reach (the touched bricks) read once
        "shift": None,
        # per reconstruction (all launches of the stage together):
        # y forward of the grids' spectra (tiles with data in, whole spectra out), then of delta_s
        "y_fwd_step": (fg + fr) * cn + na * cn + (fm if randoms else 1.0) * cn + cn,
        # y inverse of the smoothed spectra (whole spectra in, the mask's tiles out)
        "y_inv_step": na * cn * (1.0 + (fm if randoms else 1.0)),
        # binning, both catalogues: positions read by the count and by the scatter, brick-ordered copy
        # (16 B) and slot (4 B) written, each block's 128 KB histogram written and read back
        "bin_step": 44 * (n_gal + n_ran) + 2 * 131072 * (bin_blocks(n_gal) + bin_blocks(n_ran)),
        "fill_step": gb + rb + 2 * 4 * nbs3,                  # touched bricks cleared, brick counts zeroed
        # learned start on the network grid of (N/2^levels)^3 cells (c = 8^-levels of the cells):
        # restriction of delta_s and u_p (R in, c R out each; the (N/2)^3 intermediates of the two-level
        # form are not compulsory) and prolongation of the network output (c R in, R out); the three layers read delta and u_p (8 B per network cell), write and
        # read a1 and a2 (32 B each, bf16 x 16 channels) and write Delta u (4 B)
        "resample_step": (2 * 4 + 2 * 4 * 8.0 ** -levels + 4 * 8.0 ** -levels + 4) * n3,
        "cnn_fwd_step": (8 + 32 + 32 + 32 + 32 + 4) * n3 * 8.0 ** -levels,
    }


COPY_BYTES = 1 << 30
PROFILE = os.path.join(ROOT, "profiles", "survey512_kernels.md")


def kernel_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1504_02591_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel sources changed after the counters were taken."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    block = text.split("```\nsource ")[-1].split("```")[0].split("\n")
    if block[0].strip() != kernel_source_hash():
        return None
    for line in block[1:]:
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic" and parts[1] == "k_" + kernel:
            return int(parts[2])
    return None


def measure_copy_bandwidth(torch, dev, reps=10):
    """Device-to-device copy of 1 GiB (torch's copy kernel): read + write bytes per second."""
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * COPY_BYTES * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def time_oracle_sample(n, tol, max_iter, full=False):
    """The whole FP64 oracle pipeline (deposit of galaxies and randoms, smoothing, mask, overdensity,
    passes to eps <= tol, shift of both catalogues) on the survey workload shrunk by 2 per axis:
    (n/2)^3 grid over half the box and shell, so the same cell size and 1/8 of the cells and objects;
    full=True runs the workload itself (n^3, minutes).  Returns (seconds, passes, objects, threads, the
    catalogue, the oracle's result)."""
    from oracle import recon_oracle as O
    from synth import generators as G
    cat = G.config2(n=n, scale=n / 512.0) if full else G.config2(n=n // 2, scale=0.5, seeds=(911, 912, 913))
    t0 = time.perf_counter()
    res = O.reconstruct(cat.gal_pos, None, cat.ran_pos, None, cat.n, cat.box_len, cat.origin, cat.observer,
                        cat.bias, cat.growth, cat.smooth_r, cat.mask_tau, tol=tol, max_iter=max_iter,
                        log=(lambda m: print(f"[bench] {m} ({time.perf_counter() - t0:.1f}s)", file=sys.stderr,
                                             flush=True)) if full else None)
    dt = time.perf_counter() - t0
    return dt, res["passes"], int(cat.gal_pos.shape[0] + cat.ran_pos.shape[0]), O.WORKERS, cat, res


def gpu_error_vs_oracle(cat, ref, torch, native, dev):
    """The GPU path on the oracle's timed sample (plain start, the oracle's pass count): Psi relative L2
    error, eps history agreement and the largest displacement difference against the oracle's result."""
    import numpy as np
    plan = native.plan_for(cat)
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    ran = torch.from_numpy(cat.ran_pos).to(dev)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve()
    rc, iters, eps = plan.iterate(ref["passes"], 0.0)
    psi = plan.psi()[0].cpu().numpy().astype(np.float64)
    dg = plan.shift(native.GAL, gal).cpu().numpy()
    dr = plan.shift(native.RAN, ran).cpu().numpy()
    plan.close()
    e_psi = float(np.linalg.norm(psi - ref["psi"]) / np.linalg.norm(ref["psi"]))
    e_eps = float(np.max(np.abs(np.asarray(eps[0]) - np.asarray(ref["eps"])) / np.asarray(ref["eps"])))
    e_disp = float(max(np.abs(dg - ref["disp_g"]).max(), np.abs(dr - ref["disp_r"]).max()))
    return {"workload": f"the oracle's timed sample ({cat.n}^3, {cat.gal_pos.shape[0] + cat.ran_pos.shape[0]} "
                        f"objects), plain start, {ref['passes']} passes",
            "psi_rel_l2": e_psi, "eps_max_rel": e_eps, "disp_max_abs_mpc_h": e_disp,
            "bar": {"psi_rel_l2": 1e-5, "disp_max_abs_mpc_h": 1e-4}}


def _one_fft_thread():
    from synth import generators as G
    G.WORKERS = 1


def _batched_realisation(i):
    from synth import generators as G
    return G.config4_realisation(i)


def batched_catalogues(count):
    """Realisations of the batched workload, generated in worker processes before the GPU is used."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    cats = []
    with mp.get_context("fork").Pool(min(16, count), initializer=_one_fft_thread) as pool:
        for k, c in enumerate(pool.imap(_batched_realisation, range(count))):
            cats.append(c)
            if (k + 1) % 16 == 0:
                print(f"[bench] {k + 1}/{count} batched realisations generated", file=sys.stderr, flush=True)
    print(f"[bench] generated {count} batched realisations in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    return cats


def run_batched(args, cats, torch, native, dev):
    """The batched workload: independent 256^3 realisations (log-uniform galaxy counts, 50x randoms) in
    sub-batches of args.sub_batch through one plan: per sub-batch one deposit launch chain per catalogue
    kind over ragged offsets, batched transforms, per-realisation convergence.  Every sub-batch's
    catalogues are resident on the device before timing; one step reconstructs every realisation."""
    import numpy as np
    total = len(cats)
    sb = min(total, args.sub_batch if args.sub_batch > 0 else total)
    groups = [cats[k:k + sb] for k in range(0, total, sb)]
    if len(groups[-1]) != sb:
        sys.exit("the realisation count must be a multiple of --sub-batch")
    data = []
    for grp in groups:
        gal = torch.from_numpy(np.concatenate([c.gal_pos for c in grp])).to(dev)
        ran = torch.from_numpy(np.concatenate([c.ran_pos for c in grp])).to(dev)
        goff = torch.tensor(np.cumsum([0] + [c.gal_pos.shape[0] for c in grp]), dtype=torch.int64, device=dev)
        roff = torch.tensor(np.cumsum([0] + [c.ran_pos.shape[0] for c in grp]), dtype=torch.int64, device=dev)
        data.append((gal, ran, goff, roff))
    n_gal = sum(int(d[0].shape[0]) for d in data)
    n_ran = sum(int(d[1].shape[0]) for d in data)
    max_obj = max(int(d[1].shape[0]) for d in data)
    disp_g = torch.empty(max(int(d[0].shape[0]) for d in data), 3, dtype=torch.float32, device=dev)
    disp_r = torch.empty(max_obj, 3, dtype=torch.float32, device=dev)
    res = time_batched(args, cats, data, sb, max_obj, disp_g, disp_r, native, torch, relaxed=False)
    res["workload"] = (f"{total} realisations of 256^3 over 1500 Mpc/h in sub-batches of {sb} through one plan, "
                       f"galaxies log-uniform in [1e5, 1e6] ({n_gal} in total), 50x randoms ({n_ran}), plain start "
                       f"to eps<={args.tol:g}")
    if args.batched_relaxed:
        res["relaxed"] = time_batched(args, cats, data, sb, max_obj, disp_g, disp_r, native, torch, relaxed=True)
    return res


def time_batched(args, cats, data, sb, max_obj, disp_g, disp_r, native, torch, relaxed):
    """Timed steps of the batched workload through one plan (relaxed: the relaxed correction pass)."""
    total = len(cats)
    c0 = cats[0]
    plan = native.Plan(c0.n, c0.box_len, c0.observer, c0.bias, c0.growth, c0.smooth_r, origin=c0.origin, batch=sb,
                       mask_tau=c0.mask_tau, max_objects=max_obj, graphs=not args.no_graphs, relaxed=relaxed)
    passes, codes = [], {}

    def step():
        passes.clear()
        for gal, ran, goff, roff in data:
            plan.paint(native.GAL, gal, offsets=goff)
            plan.paint(native.RAN, ran, offsets=roff)
            plan.solve()
            rc, iters, eps = plan.iterate(args.max_iter, args.tol)
            plan.shift(native.GAL, gal, offsets=goff, out_disp=disp_g[:gal.shape[0]])
            plan.shift(native.RAN, ran, offsets=roff, out_disp=disp_r[:ran.shape[0]])
            passes.extend(iters)
            codes[rc] = codes.get(rc, 0) + 1

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    steps = max(3, args.steps // 4)
    t0 = time.perf_counter()
    for k in range(steps):
        step()
        print(f"[bench] batched step {k + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.close()
    if native.RECON_NOTCONVERGED in codes:
        sys.exit("bench: a batched realisation did not reach the tolerance")
    res = {"realisations": total, "sub_batch": sb, "steps": steps, "ms_per_step": round(1e3 * el / steps, 3),
           "realisations_per_s": round(total * steps / el, 2), "passes_min_max": [min(passes), max(passes)],
           "step_return_codes": {str(k): v for k, v in codes.items()}}
    print(f"[bench] batched{' (relaxed pass)' if relaxed else ''}: {total} realisations in sub-batches of {sb}, "
          f"{1e3 * el / steps:.2f} ms per step, passes {min(passes)}..{max(passes)}", file=sys.stderr, flush=True)
    return res


def run_precision(args):
    """The precision study: the periodic 1024^3 box of 1024^3 Zel'dovich lattice particles (L = 2000 Mpc/h,
    f = 0.76, b = 1, R = 10 Mpc/h, observer 5000 Mpc/h from the centre, mean-density overdensity) in FP32
    and with the split-bfloat16 matrix-core radix-8 stage (2 and 3 terms); every variant timed per
    reconstruction (deposit, solve, passes to eps <= tol, shift of all particles), compared with the FP32
    result at 1024^3 and with the FP64 oracle on the 128^3 sub-run of the same geometry."""
    import numpy as np
    import torch
    from oracle import recon_oracle as O
    from paper_1504_02591_amd import native
    from synth import generators as G

    def log(msg):
        print(f"[precision] {msg}", file=sys.stderr, flush=True)

    # (split-bf16 terms, relaxed pass): the FP32 and split-bf16 transforms with the paper's pass, and the
    # FP32 transforms with the relaxed pass (beta = 0.76 here, where it shortens the iteration most)
    variants = ((0, False), (2, False), (3, False), (0, True))
    names = {(0, False): "fp32", (2, False): "split_bf16_2", (3, False): "split_bf16_3", (0, True): "fp32_relaxed"}
    out = {"subrun_128": {}, "n1024": {}}
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # 128^3 sub-run against the FP64 oracle (6 fixed passes)
    sub = G.config3(128)
    refs = {relaxed: O.reconstruct(sub.gal_pos, None, None, None, sub.n, sub.box_len, sub.origin, sub.observer,
                                   sub.bias, sub.growth, sub.smooth_r, n_passes=6,
                                   relax=O.relax_weight(sub.growth, sub.bias) if relaxed else None)
            for relaxed in (False, True)}
    gsub = torch.from_numpy(sub.gal_pos).to(dev)
    for v in variants:
        plan = native.plan_for(sub, split_terms=v[0], relaxed=v[1])
        plan.paint(native.GAL, gsub)
        plan.solve()
        plan.iterate(6, 0.0)
        psi = plan.psi()[0].cpu().numpy().astype(np.float64)
        plan.close()
        ref = refs[v[1]]
        e = float(np.linalg.norm(psi - ref["psi"]) / np.linalg.norm(ref["psi"]))
        out["subrun_128"][names[v]] = {"psi_rel_l2_vs_fp64_oracle": e}
        log(f"128^3 sub-run, {names[v]}: Psi rel L2 vs FP64 oracle {e:.3e}")
    del gsub
    # the 1024^3 box
    t0 = time.perf_counter()
    cat = G.config3(1024, log=log)
    log(f"1024^3 lattice: {cat.gal_pos.shape[0]} particles in {time.perf_counter() - t0:.1f}s")
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    cat.gal_pos = None
    disp = torch.empty_like(gal)
    psi_fp32 = None
    for v in variants:
        plan = native.Plan(1024, cat.box_len, cat.observer, cat.bias, cat.growth, cat.smooth_r, randoms=False,
                           max_objects=int(gal.shape[0]), graphs=True, split_terms=v[0], relaxed=v[1])
        log(f"{names[v]}: plan of {plan.workspace.numel() / 1e9:.1f} GB")
        passes, rcs = [], []

        def step():
            plan.paint(native.GAL, gal)
            plan.solve()
            rc, iters, eps = plan.iterate(args.max_iter, args.tol)
            plan.shift(native.GAL, gal, out_disp=disp)
            passes.append(iters[0])
            rcs.append(rc)
            return eps[0]

        step()
        torch.cuda.synchronize()
        k = max(1, args.steps // 4)
        t1 = time.perf_counter()
        for _ in range(k):
            eps = step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        plan.profile_start()
        step()
        prof = plan.profile_stop()
        psi = plan.psi()[0]
        plan.close()
        del plan
        ent = {"ms_per_recon": round(1e3 * el / k, 2), "recons_per_s": round(k / el, 4), "passes": passes[-1],
               "eps": eps, "return_codes": sorted(set(rcs)),
               "z_iter_avg_launch_ms": round(prof["z_iter"][1] / prof["z_iter"][0], 4) if "z_iter" in prof else None}
        if psi_fp32 is None:
            psi_fp32 = psi
        else:
            # split-bf16: the transforms' error; relaxed: the difference of two iterates stopped at eps <= tol
            key = "psi_rel_l2_vs_fp32_paper_pass" if v[1] else "psi_rel_l2_vs_fp32"
            ent[key] = float((psi - psi_fp32).double().norm() / psi_fp32.double().norm())
            del psi
        out["n1024"][names[v]] = ent
        log(f"1024^3 {names[v]}: {ent}")
        torch.cuda.empty_cache()
    res = {"metric": "1024^3 precision study: reconstructions/s (FP32 and split-bf16 radix) and Psi rel L2",
           "value": out["n1024"]["fp32"]["recons_per_s"], "unit": "recons/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"periodic 1024^3 grid over 2000 Mpc/h, {int(gal.shape[0])} Zel'dovich lattice "
                                  f"particles, f=0.76 b=1 R=10, observer 5000 Mpc/h from the centre, mean-density "
                                  f"overdensity, passes to eps<={args.tol:g}"},
           "variants": out}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--rounds", type=int, default=5, help="interleaved timing rounds over the starts")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--starts", default="plain_relaxed,learned_relaxed,plain,ffta2,learned",
                    help="comma-separated starts to time (suffix _relaxed: the relaxed correction pass); the last "
                         "one available is the headline value")
    ap.add_argument("--weights", default=None, help="learned-start parameters (.npz, key 'params')")
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=50)
    ap.add_argument("--n", type=int, default=512, help="grid size (512 is the measured workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle on the full workload instead of the 1/8 sample (minutes)")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--no-graphs", action="store_true", help="launch the steady-state pass eagerly")
    ap.add_argument("--lognormal", action="store_true", help="lognormal transform of delta_s (Sec. 6)")
    ap.add_argument("--ngp", action="store_true", help="nearest-grid-point deposit (the paper's binning)")
    ap.add_argument("--precision", action="store_true",
                    help="run the 1024^3 precision study (FP32 vs split-bf16 radix) instead of the survey workload")
    ap.add_argument("--batched", type=int, default=0,
                    help="also time B realisations of the batched 256^3 workload (256 is the full workload)")
    ap.add_argument("--sub-batch", type=int, default=64,
                    help="realisations per plan call in the batched workload (the plan's batch)")
    ap.add_argument("--batched-only", action="store_true", help="time only the batched workload")
    ap.add_argument("--batched-relaxed", action="store_true",
                    help="also time the batched workload with the relaxed correction pass")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures a single MI355X: this build has no multi-GPU path; run with --gpus 1",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.precision:
        run_precision(args)
        return

    import numpy as np
    from synth import generators as G
    batch_cats = batched_catalogues(args.batched) if args.batched > 0 else None   # before the GPU is used
    import torch
    from paper_1504_02591_amd import native

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.batched_only:
        if not batch_cats:
            sys.exit("--batched-only needs --batched B")
        res = run_batched(args, batch_cats, torch, native, dev)
        print(json.dumps({"metric": "batched 256^3 realisations/s to 1e-3 Psi tol", "value": res["realisations_per_s"],
                          "unit": "realisations/s", "n_gpus": 1, "steps": res["steps"], "warmup": args.warmup,
                          "higher_is_better": True, "dtype": "f32", "data": "synthetic", "config": res}), flush=True)
        return
    copy_gbs = measure_copy_bandwidth(torch, dev)
    t_gen = time.perf_counter()
    cat = G.config2(n=args.n, scale=args.n / 512.0)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] generated catalogue in {t_gen:.1f}s: {cat.info['n_gal']} galaxies, "
          f"{cat.info['n_ran']} randoms", file=sys.stderr, flush=True)
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    ran = torch.from_numpy(cat.ran_pos).to(dev)
    disp_g = torch.empty_like(gal)
    disp_r = torch.empty_like(ran)

    starts = [s.strip() for s in args.starts.split(",") if s.strip()]
    for s in starts:
        try:
            start_of(s)
        except KeyError:
            sys.exit(f"unknown start {s!r}")
    net, net_levels = None, 0
    if any(start_of(s)[0] == START_NAMES["learned"] for s in starts):
        from paper_1504_02591_amd import learned
        wpath = args.weights or learned.WEIGHTS
        if os.path.exists(wpath):
            with np.load(wpath, allow_pickle=False) as z:
                net = torch.from_numpy(np.ascontiguousarray(z["params"], dtype=np.float32)).to(dev)
                net_levels = int(z["levels"]) if "levels" in z.files else (1 if "half" in z.files and bool(z["half"])
                                                                             else 0)
        else:
            print(f"[bench] no learned-start weights at {wpath}: learned start skipped", file=sys.stderr, flush=True)
            starts = [s for s in starts if start_of(s)[0] != START_NAMES["learned"]]

    def make_plan(name):
        start, relaxed = start_of(name)
        lrn = start == START_NAMES["learned"]
        return native.plan_for(cat, start_buffers=start != 0, keep_delta=lrn, cnn=lrn,
                               cnn_half=lrn and net_levels == 1, cnn_quarter=lrn and net_levels == 2,
                               graphs=not args.no_graphs, lognormal=args.lognormal, relaxed=relaxed)

    codes = {}

    def run(plan, start, steps, passes):
        eps_last = None
        for _ in range(steps):
            plan.paint(native.GAL, gal, ngp=args.ngp)
            plan.paint(native.RAN, ran, ngp=args.ngp)
            plan.solve(start, net if start == START_NAMES["learned"] else None)
            rc, iters, eps = plan.iterate(args.max_iter, args.tol)
            plan.shift(native.GAL, gal, out_disp=disp_g)
            plan.shift(native.RAN, ran, out_disp=disp_r)
            passes.append(iters[0])
            codes[rc] = codes.get(rc, 0) + 1     # host-side count: every step's return code is kept
            eps_last = eps[0]
        return eps_last  # eps history of the last step

    # The starts are timed interleaved: each of `rounds` rounds runs a block of steps of every start
    # (in an order rotated from round to round), each block bracketed by device synchronisations, so
    # that clock or thermal drift over the run falls on all starts alike.  Every start runs exactly
    # args.steps timed steps in total.
    plans = {name: make_plan(name) for name in starts}
    for name in starts:
        run(plans[name], start_of(name)[0], args.warmup, [])
    torch.cuda.synchronize()
    rounds = max(1, min(args.rounds, args.steps))
    blocks = [args.steps // rounds + (1 if r < args.steps % rounds else 0) for r in range(rounds)]
    acc = {name: {"elapsed": 0.0, "passes": [], "eps": None} for name in starts}
    for r, k in enumerate(blocks):
        for name in starts[r % len(starts):] + starts[:r % len(starts)]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eps = run(plans[name], start_of(name)[0], k, acc[name]["passes"])
            torch.cuda.synchronize()
            acc[name]["elapsed"] += time.perf_counter() - t0
            acc[name]["eps"] = eps
    if any(rc == native.RECON_NOTCONVERGED for rc in codes):
        sys.exit(f"bench: {codes[native.RECON_NOTCONVERGED]} steps did not reach eps <= {args.tol:g} within "
                 f"{args.max_iter} passes: no reconstructions/s is reported")
    results = {}
    for name in starts:
        restarts = plans[name].restarts()[0]
        plans[name].close()
        elapsed, p_, eps_last = acc[name]["elapsed"], acc[name]["passes"], acc[name]["eps"]
        results[name] = {"passes": p_[-1], "eps": eps_last, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
                         "recons_per_s": round(args.steps / elapsed, 3), "elapsed": elapsed,
                         "restarts_last_step": restarts}
        print(f"[bench] {name}: {args.steps} steps in {elapsed:.3f}s ({rounds} interleaved rounds), {p_[-1]} passes, "
              f"eps {eps_last[-1]:.3g}", file=sys.stderr, flush=True)
    del plans
    head = starts[-1]
    elapsed = results[head]["elapsed"]
    passes = [results[head]["passes"]]
    eps_last = results[head]["eps"]

    # per-kernel event timing: a separate run of the headline start, so the timed run carries no events
    prof, tiles = {}, None
    if not args.no_profile:
        start = start_of(head)[0]
        plan = make_plan(head)
        run(plan, start, 1, [])
        plan.profile_start()
        run(plan, start, args.steps, [])
        prof = plan.profile_stop()
        tiles = plan.tile_counts()[0]
        plan.close()

    ms_per_step = 1e3 * elapsed / max(args.steps, 1)
    value = args.steps / elapsed
    n_gal, n_ran = int(gal.shape[0]), int(ran.shape[0])
    bricks_g = touched_bricks(cat.gal_pos, args.n, cat.box_len)
    bricks_r = touched_bricks(cat.ran_pos, args.n, cat.box_len)
    ab = algorithmic_bytes(args.n, n_gal, n_ran, bricks_g=bricks_g, bricks_r=bricks_r, levels=max(net_levels, 1),
                           tiles=tiles, keep_delta=start_of(head)[0] == START_NAMES["learned"])
    stages = {}
    for name, (count, tot_ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        per = ab.get(name)
        if name == "z_iter" and start_of(head)[0] != START_NAMES["plain"] and per is not None:
            # the start pass and the pass after it also read (or write) the start correction field;
            # the learned start's pass reads u_p (one real field) instead of the two state-Y spectra
            r = args.n ** 3 * 4
            per_step = per * count / args.steps + 2 * r
            if start_of(head)[0] == START_NAMES["learned"]:
                per_step += r - per / 2
        elif name == "y_fanout":
            # one full fan-out per reconstruction (the output), the rest combined
            per_step = (per * (count - args.steps) + ab["y_fanout_full"] * args.steps) / args.steps
        elif name == "z_final" and start_of(head)[0] == START_NAMES["learned"]:
            # u_p of the start (combined state) plus the output
            per_step = ab["z_final_u"] + per
        elif name == "paint":
            per_step = 12 * (n_gal + n_ran) + ab["paint_grids"]
        elif name == "shift":
            per_step = 24 * (n_gal + n_ran) + 12 * BRICK ** 3 * (bricks_g + bricks_r)
        elif name + "_step" in ab:
            per_step = ab[name + "_step"]
        else:
            per_step = None if per is None else per * count / args.steps
        ent = {"launches_per_step": count / args.steps, "ms_per_step": tot_ms / args.steps,
               "avg_launch_ms": tot_ms / count}
        if per_step is not None and tot_ms > 0:
            ent["algorithmic_GBs"] = per_step * args.steps / (tot_ms * 1e-3) / 1e9
            ent["frac_hbm_peak"] = ent["algorithmic_GBs"] / HBM_PEAK_GBS
        stages[name] = ent
    roofline = None
    candidates = [k for k in stages if ab.get(k) is not None]
    if candidates:
        dom = max(candidates, key=lambda k: stages[k]["ms_per_step"])
        avg_s = stages[dom]["avg_launch_ms"] * 1e-3
        per_launch = stages[dom]["algorithmic_GBs"] * 1e9 * avg_s     # launch-averaged algorithmic bytes
        ach = per_launch / avg_s / 1e9
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dom) if args.n == 512 else None,
                    "algorithmic_bytes_per_launch": int(round(per_launch)), "avg_launch_ms": round(avg_s * 1e3, 4)}

    cpu = vs_oracle = None
    if not args.no_cpu_baseline:
        t_s, p_s, m_s, workers, s_cat, s_ref = time_oracle_sample(args.n, args.tol, args.max_iter, full=args.cpu_full)
        vs_oracle = gpu_error_vs_oracle(s_cat, s_ref, torch, native, dev)
        del s_cat, s_ref
        print(f"[bench] GPU vs oracle on the sample: psi rel L2 {vs_oracle['psi_rel_l2']:.2e}, displacement "
              f"{vs_oracle['disp_max_abs_mpc_h']:.2e} Mpc/h", file=sys.stderr, flush=True)
        if args.cpu_full:
            cpu = {"value": 1.0 / t_s, "unit": "recons/s", "cores": workers, "kind": "oracle",
                   "host_cpu_count": os.cpu_count(),
                   "sample": f"the FP64 oracle's whole reconstruction (deposit, smoothing, mask, overdensity, "
                             f"{p_s} passes to eps<={args.tol:g}, shift) of the full workload ({args.n}^3, {m_s} "
                             f"objects) took {t_s:.1f}s with scipy.fft on {workers} threads"}
        else:
            cpu = {"value": 1.0 / (8.0 * t_s), "unit": "recons/s", "cores": workers, "kind": "oracle",
                   "host_cpu_count": os.cpu_count(),
                   "sample": f"the FP64 oracle's whole reconstruction (deposit, smoothing, mask, overdensity, {p_s} "
                             f"passes to eps<={args.tol:g}, shift) of the survey workload shrunk 2x per axis "
                             f"({args.n // 2}^3 grid, same cell size, {m_s} objects) took {t_s:.1f}s with "
                             f"scipy.fft on {workers} threads; value = 1/(8 x that), i.e. scaled by the 8x cells "
                             f"and objects of the full workload (the transforms' extra log factor is ignored; "
                             f"--cpu-full times the full workload)"}

    batched = run_batched(args, batch_cats, torch, native, dev) if batch_cats else None

    out = {
        "metric": "512^3 recons/s to 1e-3 Psi tol, learned vs plain start; % HBM roofline",
        "value": round(value, 3), "unit": "recons/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"survey-like {args.n}^3 grid over {cat.box_len:g} Mpc/h, observer at the box "
                               f"centre, {n_gal} galaxies in a 2.5 sr cone shell "
                               f"{cat.info['r_min']:g}-{cat.info['r_max']:g} Mpc/h, {n_ran} randoms (50x), "
                               f"b=2 f=0.74 R=15, {head} start to eps<={args.tol:g}"
                               + (", lognormal delta" if args.lognormal else "") + (", NGP deposit" if args.ngp else ""),
                   "n": args.n, "start": head, "tol": args.tol, "passes": passes[-1], "eps": eps_last,
                   "touched_bricks": {"galaxies": bricks_g, "randoms": bricks_r, "of": (args.n // BRICK) ** 3},
                   "setup_tiles": None if tiles is None else {"galaxy_grid": tiles[0], "random_grid": tiles[1],
                                                               "inside_mask": tiles[2], "of": tiles[3]}},
        "starts": {k: {kk: vv for kk, vv in v.items() if kk != "elapsed"} for k, v in results.items()},
        "step_return_codes": {str(k): v for k, v in codes.items()},
        # starts named *_relaxed run the relaxed correction pass, an option beyond the paper (its fixed point)
        "relaxed_pass": "D_{n+1} = (1 - w) D_n + w (D_s + f div[(Psi_n . r) r]), w = 2/(2 + f/b); the first pass "
                        "after the learned start is the paper's pass",
        # the paper's own figures for this method (Sec. 5.2, Tables 2-3), as context: correction passes to
        # convergence of the mean radial ratio against the true field on a BOSS DR11 CMASS mock (NGP, 512^3,
        # L = 3500 Mpc/h, R = 10 Mpc/h, b = 1.87) and an N-body box (128^3, L = 768 Mpc/h); no timings or
        # hardware are given.  This build stops on eps_n <= tol instead (the true field is unknown)
        "paper": {"passes_plain_start": {"mock": 6, "nbody": 4}, "passes_rsd_corrected_start": {"mock": 2, "nbody": 2},
                  "timings": None},
        "roofline": roofline,
        "copy_GBs": round(copy_gbs, 1),
        "cpu_baseline": cpu,
        # this run's error against the oracle, on the oracle's timed sample (the same catalogue generator)
        "vs_oracle": vs_oracle,
        "stages": stages,
    }
    if batched:
        out["batched"] = batched
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
