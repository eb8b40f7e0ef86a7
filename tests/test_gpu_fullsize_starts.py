"""The benchmarked starts at full size against the FP64 oracle, and what the trained network gains.

Survey-like catalogue on the 512^3 grid over 3500 Mpc/h (observer at the centre, 2.5 sr cone shell
1100-1800 Mpc/h, about 7e5 galaxies and 3.5e7 randoms, b = 2, f = 0.74, R = 15) in the plan
configuration the benchmark times: brick-binned deposit, steady-state pass replayed as a HIP graph,
start buffers, and for the learned start the committed network parameters evaluated on their
network grid (128^3 for the committed quarter-grid network: two-field slab restrictions, BF16 MFMA
layers, prolongations), followed by the learned start pass and the pass that finishes its eps_1.  Fixed pass counts, against the oracle's plain FP64
definition of every step (the network with the same bf16 roundings as the kernels).

The gain test runs a held-out realisation (seeds of the network's held-out set, never trained on)
with the plain, FFTA-2 (eq. approx2) and learned starts to eps <= 1e-3 and checks that the learned
start needs fewer correction passes (Sec. 5.1 iteration) than either.
"""
import functools
import time

import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C
from oracle import recon_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu

PSI_TOL = 1e-5
DISP_TOL = 1e-4


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def log(msg):
    print(msg, flush=True)


@functools.lru_cache(maxsize=1)
def survey():
    t0 = time.perf_counter()
    cat = G.config2()
    log(f"catalogue: {cat.gal_pos.shape[0]} galaxies, {cat.ran_pos.shape[0]} randoms "
        f"({time.perf_counter() - t0:.1f}s)")
    return cat


@functools.lru_cache(maxsize=1)
def oracle_base():
    """Oracle deposit grids, overdensity and plain-start radial displacement of the survey catalogue."""
    cat = survey()
    t0 = time.perf_counter()
    grid_g = O.paint(cat.gal_pos, None, cat.n, cat.box_len, cat.origin)
    grid_r = O.paint(cat.ran_pos, None, cat.n, cat.box_len, cat.origin)
    delta = O.overdensity(grid_g, grid_r, cat.box_len, cat.smooth_r, cat.mask_tau)
    rhat = O.line_of_sight(cat.n, cat.box_len, cat.origin, cat.observer)
    psi_p = O.psi_from_density(O.fwd(delta), cat.n, cat.box_len, cat.bias)
    u_p = np.sum(psi_p * rhat, axis=0)
    del psi_p
    log(f"oracle deposit, overdensity, plain start: {time.perf_counter() - t0:.1f}s on {O.WORKERS} threads")
    return grid_g, grid_r, delta, rhat, u_p


def weights():
    from paper_1504_02591_amd import learned
    with np.load(learned.WEIGHTS, allow_pickle=False) as z:
        levels = int(z["levels"]) if "levels" in z.files else (1 if bool(z["half"]) else 0)
        return np.ascontiguousarray(z["params"], dtype=np.float32), levels


def gpu_run(native, cat, start, chunks, net=None, levels=1):
    """The benchmark's plan; passes in chunks (one iterate call each), Psi after every chunk, then the
    shift of both catalogues and the deposit grids."""
    dev = torch.device("cuda", 0)
    lrn = start == native.START_LEARNED
    plan = native.plan_for(cat, keep_delta=lrn, start_buffers=start != native.START_PLAIN, cnn=lrn,
                           cnn_half=lrn and levels == 1, cnn_quarter=lrn and levels == 2, graphs=True)
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    ran = torch.from_numpy(cat.ran_pos).to(dev)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(start, None if net is None else torch.from_numpy(net).to(dev))
    out, eps_all, total = {"psi": {}}, [], 0
    for k in chunks:
        rc, iters, eps = plan.iterate(k, 0.0)
        assert rc == native.RECON_OK
        total += k
        eps_all += eps[0]
        out["psi"][total] = plan.psi()[0].cpu().numpy()
    out["eps"] = eps_all
    out["restarts"] = plan.restarts()[0]
    out["disp_g"] = plan.shift(native.GAL, gal).cpu().numpy()
    out["disp_r"] = plan.shift(native.RAN, ran).cpu().numpy()
    out["grid_g"] = plan.grid(native.GAL)[0].cpu().numpy()
    out["grid_r"] = plan.grid(native.RAN)[0].cpu().numpy()
    plan.close()
    return out


def check_shifts(g, psi_ref, cat, label):
    e_g = float(np.abs(g["disp_g"] - O.shift(psi_ref, cat.gal_pos, cat.box_len, cat.origin, cat.observer,
                                             cat.growth, True)).max())
    e_r = float(np.abs(g["disp_r"] - O.shift(psi_ref, cat.ran_pos, cat.box_len, cat.origin, cat.observer,
                                             cat.growth, False)).max())
    log(f"{label}: displacement max |d| galaxies {e_g:.2e}, randoms {e_r:.2e} Mpc/h")
    assert e_g <= DISP_TOL and e_r <= DISP_TOL


@pytest.mark.timeout(1200)
def test_learned_start_512_benchmark_configuration(gpu_lib):
    from paper_1504_02591_amd import native
    cat = survey()
    net, levels = weights()
    assert levels >= 1, "the committed network runs on a coarser grid than the solver's"
    g = gpu_run(native, cat, native.START_LEARNED, (2, 3), net, levels)
    log(f"GPU learned start: eps {g['eps']}, restarts {g['restarts']}")
    assert g["restarts"] == 0
    grid_g, grid_r, delta, rhat, u_p = oracle_base()
    assert np.array_equal(g["grid_g"], grid_g), "galaxy grid not bit-exact"
    assert np.array_equal(g["grid_r"], grid_r), "random grid not bit-exact"
    t0 = time.perf_counter()
    rhat_c = O.line_of_sight(cat.n >> levels, cat.box_len, cat.origin, cat.observer)
    du = C.coarse_grid_correction(net.astype(np.float64), delta, u_p, rhat_c, levels, bf16_mode=True,
                                  conv_fn=C.conv_loops)
    del rhat_c
    log(f"oracle network on the {cat.n >> levels}^3 grid: {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    ref = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth, n_passes=5,
                              start=O.START_LEARNED, start_correction=du, rhat=rhat, keep=(2,))
    log(f"oracle 5 passes: {time.perf_counter() - t0:.1f}s; eps {ref['eps']}")
    e2 = rel_l2(g["psi"][2], ref["psi_at"][2])
    e5 = rel_l2(g["psi"][5], ref["psi"])
    log(f"512^3 learned start: psi rel L2 after 2 passes {e2:.2e}, after 5 passes {e5:.2e}")
    assert e2 <= 1e-4
    assert e5 <= PSI_TOL
    np.testing.assert_allclose(g["eps"], ref["eps"], rtol=1e-3, atol=1e-6)
    check_shifts(g, ref["psi"], cat, "512^3 learned start, 5 passes")


@pytest.mark.timeout(1200)
def test_ffta2_start_512_benchmark_configuration(gpu_lib):
    from paper_1504_02591_amd import native
    cat = survey()
    g = gpu_run(native, cat, native.START_FFTA2, (2,))
    grid_g, grid_r, delta, rhat, _ = oracle_base()
    assert np.array_equal(g["grid_g"], grid_g) and np.array_equal(g["grid_r"], grid_r)
    t0 = time.perf_counter()
    ref = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth, n_passes=2,
                              start=O.START_FFTA2, rhat=rhat)
    log(f"oracle FFTA-2, 2 passes: {time.perf_counter() - t0:.1f}s")
    e = rel_l2(g["psi"][2], ref["psi"])
    log(f"512^3 FFTA-2 start: psi rel L2 after 2 passes {e:.2e}; eps gpu {g['eps']} oracle {ref['eps']}")
    assert e <= PSI_TOL
    np.testing.assert_allclose(g["eps"], ref["eps"], rtol=1e-4, atol=1e-6)
    check_shifts(g, ref["psi"], cat, "512^3 FFTA-2 start, 2 passes")


@pytest.mark.timeout(600)
def test_trained_network_saves_passes_on_held_out_realisation(gpu_lib):
    from paper_1504_02591_amd import native
    from paper_1504_02591_amd import learned
    i = 1          # held-out set: seeds 60000 + 3 i .. (training used 50000 + 3 i ..)
    base = learned.TEST_SEED
    cat = G.config2(seeds=(base + 3 * i, base + 3 * i + 1, base + 3 * i + 2))
    net, levels = weights()
    dev = torch.device("cuda", 0)
    gal = torch.from_numpy(cat.gal_pos).to(dev)
    ran = torch.from_numpy(cat.ran_pos).to(dev)
    res = {}
    for name, start in (("plain", native.START_PLAIN), ("ffta2", native.START_FFTA2),
                        ("learned", native.START_LEARNED)):
        lrn = start == native.START_LEARNED
        plan = native.plan_for(cat, keep_delta=lrn, start_buffers=start != native.START_PLAIN, cnn=lrn,
                               cnn_half=lrn and levels == 1, cnn_quarter=lrn and levels == 2, graphs=True)
        netd = torch.from_numpy(net).to(dev) if lrn else None
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.paint(native.GAL, gal)
            plan.paint(native.RAN, ran)
            plan.solve(start, netd)
            rc, iters, eps = plan.iterate(30, 1e-3)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        assert rc == native.RECON_OK
        res[name] = dict(passes=iters[0], eps=eps[0], psi=plan.psi()[0].cpu().numpy(), ms=1e3 * min(times),
                         restarts=plan.restarts()[0])
        plan.close()
        log(f"held-out realisation, {name} start: {iters[0]} passes, eps {eps[0][-1]:.2e}, "
            f"{res[name]['ms']:.2f} ms (paint to converged Psi, best of 3)")
    assert res["learned"]["restarts"] == 0
    assert res["learned"]["passes"] < res["plain"]["passes"]
    assert res["learned"]["passes"] < res["ffta2"]["passes"]
    # every start converges to the same fixed point: the stopping iterates agree to about the tolerance
    d = rel_l2(res["learned"]["psi"], res["plain"]["psi"])
    log(f"learned vs plain converged Psi: rel L2 {d:.2e}")
    assert d < 3e-3
