"""Training and evaluation of the learned starting displacement (recon_cnn.h).

Targets come from the reconstruction itself: for each synthetic survey
realisation the plain start is iterated to a tight tolerance on the GPU, and the
network learns the radial correction Delta u* = u_inf - u_p between the
converged and the plain-start radial displacement.  Training runs entirely in
the library's own kernels (recon_cnn_train_step: forward, backward and Adam).

By default the network runs on the (n/2)^3 grid (RECON_CNN_HALF): training
realisations are survey-like catalogues of the 512^3 workload's geometry, solved
at 512^3, and delta_s, u_p and the target are restricted to the 256^3 network
grid; inference restricts the 512^3 inputs the same way and prolongs Delta u.
--levels 2 puts it on the (n/4)^3 grid (RECON_CNN_QUARTER, restricted twice),
--levels 0 on the solver grid itself.  Every realisation (galaxies
only) shares one random catalogue, as a survey's realisations share its randoms.  Test
realisations use other seeds.

    python -m paper_1504_02591_amd.learned --train 64 --steps 1500 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np
import torch

from . import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "learned_start.npz")
TRAIN_SEED, TEST_SEED = 50000, 60000


def _catalogue(args):
    """Galaxies of one survey realisation (no randoms: every realisation shares one random catalogue).

    The linear field is drawn on a gen_n^3 grid over the benchmark box; the catalogue is reconstructed
    on the n^3 grid."""
    import dataclasses
    from synth import generators as G
    i, train, n, gen_n = args
    base = TRAIN_SEED if train else TEST_SEED
    cat = G.config2(n=gen_n, scale=n / 512.0, seeds=(base + 3 * i, base + 3 * i + 1, base + 3 * i + 2),
                    ran_factor=0)
    return dataclasses.replace(cat, n=n)


def _randoms(n):
    """The shared random catalogue (50x the expected galaxy count, same survey mask)."""
    from synth import generators as G
    # the randoms depend on the field only through the galaxy count: a coarse field suffices
    return G.config2(n=64, scale=n / 512.0, seeds=(TRAIN_SEED - 3, TRAIN_SEED - 2, TRAIN_SEED - 1)).ran_pos


def _init_worker(threads):
    from synth import generators as G
    G.WORKERS = threads


def catalogue_pool(workers, threads=None):
    """Worker processes for host-side catalogue generation (FFT threads split between them);
    create before the GPU is touched."""
    t = threads if threads is not None else max(1, 16 // max(workers, 1))
    return mp.get_context("fork").Pool(workers, initializer=_init_worker, initargs=(t,))


def _levels(half):
    """Coarsening levels of the network grid (True: 1, False: 0, or the level count itself)."""
    return int(half) if isinstance(half, bool) else int(half)


def _plan_flags(levels):
    return dict(cnn_half=levels == 1, cnn_quarter=levels == 2)


def targets(cat, ran, half=True, tol=1e-6, max_iter=200):
    """(delta_s, u_p, Delta u*, passes) for one galaxy catalogue and the shared randoms (device
    tensor) on the network grid, from the plain start iterated to tol on the GPU; the fields are
    restricted half (True = 1, or a level count) times."""
    dev = torch.device("cuda", torch.cuda.current_device())
    plan = native.plan_for(cat, keep_delta=True, max_objects=max(cat.gal_pos.shape[0], ran.shape[0]))
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    del gal
    plan.solve(native.START_PLAIN)
    plan.iterate(0, 0.0)
    u_p = plan.radial()
    rc, iters, eps = plan.iterate(max_iter, tol)
    u_inf = plan.radial()
    delta = plan.delta()
    levels = _levels(half)
    for lv in range(levels):
        rp = plan if lv == 0 else native.Plan(cat.n >> lv, cat.box_len, cat.observer, cat.bias, cat.growth,
                                              cat.smooth_r, origin=cat.origin, randoms=False)
        delta, u_p, u_inf = rp.restrict(delta), rp.restrict(u_p), rp.restrict(u_inf)
        if lv > 0:
            rp.close()
    plan.close()
    return delta[0].clone(), u_p[0].clone(), (u_inf - u_p)[0].clone(), iters[0]


def init_params(seed=0):
    """He-style random weights (float32), layout W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((16, 27, 8)) * np.sqrt(2.0 / (27 * 5))
    w1[:, :, 5:] = 0.0
    w2 = rng.standard_normal((16, 27, 16)) * np.sqrt(2.0 / (27 * 16))
    w3 = rng.standard_normal((1, 27, 16)) * np.sqrt(1.0 / (27 * 16))
    th = np.concatenate([w1.ravel(), np.zeros(16), w2.ravel(), np.zeros(16), w3.ravel(), np.zeros(1)])
    assert th.size == native.CNN_PARAMS
    return th.astype(np.float32)


def train(data, geom, steps, lr, seed=0, log_every=50, params=None, state=None, half=True, total=None):
    """Adam on single realisations drawn at random; cosine learning-rate decay over `total` steps (default:
    this call's steps).  Returns (params, state, log).

    The realisation of step s is drawn from a generator seeded by (seed, s) and the rate is a function of s
    and total, so a run resumed from its saved state (params, Adam moments, step count, total) continues
    exactly as an uninterrupted run would: the same parameters bit for bit."""
    dev = torch.device("cuda", torch.cuda.current_device())
    m = data[0][0].shape[-1]
    levels = _levels(half)
    plan = native.Plan(m << levels, geom["box_len"], geom["observer"], geom["bias"], geom["growth"],
                       geom["smooth_r"], origin=geom["origin"], randoms=False, cnn=True, **_plan_flags(levels))
    th = torch.from_numpy(init_params(seed) if params is None else params).to(dev)
    m = torch.zeros_like(th) if state is None else torch.from_numpy(state["m"]).to(dev)
    v = torch.zeros_like(th) if state is None else torch.from_numpy(state["v"]).to(dev)
    step0 = 0 if state is None else int(state["step"])
    if total is None:
        total = int(state["total"]) if state is not None and "total" in state else step0 + steps
    log = []
    for s in range(step0 + 1, step0 + steps + 1):
        k = int(np.random.default_rng([seed, s]).integers(len(data)))
        d, u, t = data[k][:3]
        frac = min((s - 1) / max(total - 1, 1), 1.0)
        rate = lr * 0.5 * (1.0 + np.cos(np.pi * frac))
        loss = plan.cnn_train_step(th, m, v, s, rate, d, u, t)
        if s % log_every == 0 or s == step0 + 1:
            log.append((s, loss))
            print(f"[train] step {s} loss {loss:.5e} lr {rate:.2e}", flush=True)
    plan.close()
    state = {"m": m.cpu().numpy(), "v": v.cpu().numpy(), "step": step0 + steps, "total": total}
    return th.cpu().numpy(), state, log


def save_checkpoint(path, params, state, seed, **extra):
    """Parameters, Adam moments, step count, schedule length and seed in one .npz (no pickled objects)."""
    np.savez(path, params=params, adam_m=state["m"], adam_v=state["v"], step=state["step"], total=state["total"],
             seed=seed, **extra)


def load_checkpoint(path):
    """(params, state, seed) from save_checkpoint's file; train(..., params=params, state=state, seed=seed)
    continues the run."""
    with np.load(path, allow_pickle=False) as z:
        state = {"m": z["adam_m"].copy(), "v": z["adam_v"].copy(), "step": int(z["step"])}
        if "total" in z.files:
            state["total"] = int(z["total"])
        return z["params"].copy(), state, int(z["seed"])


def passes_to_tol(cat, ran, start, params=None, tol=1e-3, max_iter=60, half=True):
    dev = torch.device("cuda", torch.cuda.current_device())
    lrn = start == native.START_LEARNED
    levels = _levels(half) if lrn else 0
    plan = native.plan_for(cat, keep_delta=lrn, start_buffers=start != native.START_PLAIN, cnn=lrn,
                           max_objects=max(cat.gal_pos.shape[0], ran.shape[0]), **_plan_flags(levels))
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(start, None if params is None else torch.from_numpy(params).to(dev))
    rc, iters, eps = plan.iterate(max_iter, tol)
    plan.close()
    return iters[0], eps[0]


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--train", type=int, default=64, help="training realisations")
    ap.add_argument("--test", type=int, default=3, help="held-out realisations")
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--n", type=int, default=512, help="solver grid of the realisations")
    ap.add_argument("--gen-n", type=int, default=256, help="grid of the training realisations' linear fields")
    ap.add_argument("--levels", type=int, default=1, choices=(0, 1, 2),
                    help="network grid n / 2^levels (0: the solver grid, 1: (n/2)^3, 2: (n/4)^3)")
    ap.add_argument("--workers", type=int, default=16, help="catalogue generation processes")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    half = args.levels
    pool = catalogue_pool(args.workers)          # forked before the GPU is initialised
    t0 = time.time()
    # held-out realisations are drawn like the benchmark's (field on the solver grid), in the background
    test_jobs = [pool.apply_async(_catalogue, ((i, False, args.n, args.n),)) for i in range(args.test)]
    ran_host = pool.apply_async(_randoms, (args.n,)).get()
    torch.cuda.set_device(0)
    ran = torch.from_numpy(ran_host).cuda()
    print(f"[train] shared randoms: {ran.shape[0]} in {time.time() - t0:.1f}s", flush=True)
    data, geom, passes = [], None, []
    for k, cat in enumerate(pool.imap(_catalogue, [(i, True, args.n, args.gen_n) for i in range(args.train)])):
        if geom is None:
            geom = dict(box_len=cat.box_len, observer=cat.observer, bias=cat.bias, growth=cat.growth,
                        smooth_r=cat.smooth_r, origin=cat.origin)
        d = targets(cat, ran, half)
        data.append(d[:3])
        passes.append(d[3])
        if (k + 1) % 8 == 0:
            print(f"[train] {k + 1} targets after {time.time() - t0:.1f}s; plain passes to 1e-6: {passes[-8:]}",
                  flush=True)
    tests = [j.get() for j in test_jobs]
    pool.close()
    pool.join()
    t0 = time.time()
    params, state, log = train(data, geom, args.steps, args.lr, args.seed, half=half)
    t_train = time.time() - t0
    print(f"[train] {args.steps} steps in {t_train:.1f}s", flush=True)
    del data
    torch.cuda.empty_cache()
    res = {"plain": [], "ffta2": [], "learned": []}
    for c in tests:
        res["plain"].append(passes_to_tol(c, ran, native.START_PLAIN)[0])
        res["ffta2"].append(passes_to_tol(c, ran, native.START_FFTA2)[0])
        res["learned"].append(passes_to_tol(c, ran, native.START_LEARNED, params, half=half)[0])
    print("[train] held-out passes to 1e-3:", json.dumps(res), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    save_checkpoint(args.out, params, state, args.seed,
                    loss=np.array(log, dtype=np.float64), train=args.train, n=args.n, half=half == 1, levels=half,
                    eval=json.dumps(res))
    print(json.dumps({"out": args.out, "train_seconds": t_train, "final_loss": log[-1][1], "eval": res}), flush=True)


if __name__ == "__main__":
    main()
