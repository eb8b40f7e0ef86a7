"""recon_plan_noalloc (the plan on the library's own device scratch) against recon_plan.

Two no-allocation plans in a row on one GPU, the second with a smaller input, each compared with
a plan on a caller workspace running the same calls: deposit grids, displacement field, convergence
norms and shifts must be identical (the same kernels run on other memory).  The first plan is stale
once the second holds the scratch; oversized parameters and pass graphs are refused.
"""
import numpy as np
import pytest
import torch

from synth import generators as G

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def run(native, cat, noalloc, passes=3):
    plan = native.plan_for(cat, noalloc=noalloc)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve()
    rc, iters, eps = plan.iterate(passes, 0.0)
    out = dict(rc=rc, iters=iters, eps=eps, psi=plan.psi().cpu().numpy(), grid_g=plan.grid(native.GAL).cpu().numpy(),
               grid_r=plan.grid(native.RAN).cpu().numpy(), disp_g=plan.shift(native.GAL, gal).cpu().numpy(),
               disp_r=plan.shift(native.RAN, ran).cpu().numpy())
    return plan, out


def same(a, b):
    for k in ("iters", "eps"):
        assert a[k] == b[k], k
    for k in ("psi", "grid_g", "grid_r", "disp_g", "disp_r"):
        assert np.array_equal(a[k], b[k]), k


def test_noalloc_plan_equals_workspace_plan_twice(gpu_lib):
    from paper_1504_02591_amd import native
    big = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 61, 62, ran_factor=3, bias=1.2, smooth_r=20.0)
    small = G.lattice_box(16, 400.0, (-300.0, 200.0, 100.0), 0.6, 63, 64, ran_factor=2, bias=1.5, smooth_r=30.0)
    print(f"no-alloc plan: 32^3 ({big.gal_pos.shape[0]} + {big.ran_pos.shape[0]} objects), then 16^3 "
          f"({small.gal_pos.shape[0]} + {small.ran_pos.shape[0]}); scratch {gpu_lib.recon_noalloc_limit()} B",
          flush=True)
    p1, a1 = run(native, big, True)
    r1, b1 = run(native, big, False)
    r1.close()
    same(a1, b1)
    p2, a2 = run(native, small, True, passes=4)
    r2, b2 = run(native, small, False, passes=4)
    r2.close()
    same(a2, b2)
    # the first plan no longer holds the scratch
    with pytest.raises(native.ReconError) as ei:
        p1.psi()
    assert ei.value.code == native.RECON_ESTATE
    p1.close()
    p2.close()


def test_noalloc_plan_refuses_what_it_cannot_hold(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 61, 62, ran_factor=3, bias=1.2, smooth_r=20.0)
    with pytest.raises(native.ReconError) as ei:
        native.plan_for(cat, noalloc=True, max_objects=1 << 31)     # binning copy far beyond the scratch
    assert ei.value.code == native.RECON_ENOMEM
    with pytest.raises(native.ReconError) as ei:
        native.plan_for(cat, noalloc=True, graphs=True)
    assert ei.value.code == native.RECON_EINVAL
