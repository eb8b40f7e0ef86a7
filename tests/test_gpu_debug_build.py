"""The library built with its device bounds checks (RECON_DEBUG) on the hot path's configurations.

Every index the checked helpers form (transform loads and stores, z staging, the deposit's grid
atomics, Psi writes and the shift's gathers) must fall inside its array on valid inputs: the debug
build counts any that do not (and skips the access) and must count none, while producing the
release build's results.
"""
import numpy as np
import pytest
import torch

from synth import generators as G

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def run(native, lib, cat, start, net, batch_cats=None):
    kw = dict(start_buffers=start != 0, keep_delta=True, graphs=True)
    if start == native.START_LEARNED:
        kw.update(cnn=True, cnn_half=True)
    plan = native.plan_for(cat, lib=lib, **kw)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(start, None if net is None else to_dev(net))
    rc, iters, eps = plan.iterate(4, 0.0)
    out = [plan.psi().cpu().numpy(), plan.grid(native.GAL).cpu().numpy(), plan.grid(native.RAN).cpu().numpy(),
           plan.shift(native.GAL, gal).cpu().numpy(), plan.shift(native.RAN, ran).cpu().numpy(),
           plan.shift(native.RAN, ran.clone()).cpu().numpy(), np.array(eps[0])]
    plan.close()
    return out


def test_debug_build_finds_no_out_of_bounds_index(gpu_lib):
    from oracle import cnn_oracle as C
    from paper_1504_02591_amd import native
    assert gpu_lib.recon_debug_violations(0) == -1          # the release build has no checks
    dbg = native.load(native.debug_lib_path())
    assert dbg.recon_debug_violations(1) >= 0
    net = C.init_params(3).astype(np.float32)
    cases = [(G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 91, 92, ran_factor=3, bias=1.2, smooth_r=20.0),
              native.START_LEARNED, net),
             (G.config2(n=128, scale=0.25, seeds=(93, 94, 95)), native.START_FFTA2, None),
             (G.config2(n=64, scale=0.125, seeds=(96, 97, 98)), native.START_PLAIN, None)]
    for cat, start, th in cases:
        got = run(native, dbg, cat, start, th)
        assert dbg.recon_debug_violations(0) == 0, f"out-of-bounds index at n={cat.n}, start {start}"
        ref = run(native, None, cat, start, th)
        for k, (a, b) in enumerate(zip(got, ref)):
            if a.dtype == np.int64:
                assert np.array_equal(a, b), k
            else:
                # the checks change the compiled code around the transforms, so FP32 contractions may differ
                e = np.linalg.norm(a.astype(np.float64) - b) / max(np.linalg.norm(b.astype(np.float64)), 1e-30)
                assert e < 1e-6, (k, e)
        print(f"debug build n={cat.n} start {start}: no out-of-bounds index; results as the release build",
              flush=True)
