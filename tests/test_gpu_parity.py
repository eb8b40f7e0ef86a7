"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Bars: int64 deposit grids bit-exact; Psi within 1e-5 relative L2 (all cells,
three components); displacements within 1e-4 Mpc/h max-abs; convergence norms
within 1e-5 absolute.  Parity runs use fixed pass counts.
"""
import math

import numpy as np
import pytest
import torch

from oracle import recon_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu

PSI_TOL = 1e-5
DISP_TOL = 1e-4


def dev():
    return torch.device("cuda", 0)


def to_dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def gpu_catalogue_run(native, cat, n_passes, start=0, keep_delta=True, tol=0.0, lognormal=False):
    plan = native.plan_for(cat, keep_delta=keep_delta, start_buffers=start != 0, lognormal=lognormal)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal, to_dev(cat.gal_w))
    if ran is not None:
        plan.paint(native.RAN, ran, to_dev(cat.ran_w))
    plan.solve(start)
    rc, iters, eps = plan.iterate(n_passes, tol)
    out = dict(rc=rc, iters=iters[0], eps=eps[0], psi=plan.psi()[0].cpu().numpy(),
               grid_g=plan.grid(native.GAL)[0].cpu().numpy(),
               disp_g=plan.shift(native.GAL, gal).cpu().numpy())
    if ran is not None:
        out["grid_r"] = plan.grid(native.RAN)[0].cpu().numpy()
        out["disp_r"] = plan.shift(native.RAN, ran).cpu().numpy()
    if keep_delta:
        out["delta"] = plan.delta()[0].cpu().numpy()
    plan.close()
    return out


def oracle_catalogue_run(cat, n_passes, start=0, log_transform=False):
    return O.reconstruct(cat.gal_pos, cat.gal_w, cat.ran_pos, cat.ran_w, cat.n, cat.box_len, cat.origin,
                         cat.observer, cat.bias, cat.growth, cat.smooth_r, cat.mask_tau, n_passes=n_passes,
                         start=start, log_transform=log_transform)


def compare_full(g, r, label):
    assert np.array_equal(g["grid_g"], r["grid_g"]), f"{label}: galaxy grid not bit-exact"
    if "grid_r" in g and r["grid_r"] is not None:
        assert np.array_equal(g["grid_r"], r["grid_r"]), f"{label}: random grid not bit-exact"
    e_psi = rel_l2(g["psi"], r["psi"])
    e_dg = float(np.abs(g["disp_g"] - r["disp_g"]).max())
    print(f"{label}: psi relL2={e_psi:.2e} disp_g max={e_dg:.2e}", flush=True)
    assert e_psi <= PSI_TOL, f"{label}: psi rel L2 {e_psi}"
    assert e_dg <= DISP_TOL, f"{label}: galaxy displacement {e_dg}"
    if "disp_r" in g and "disp_r" in r:
        e_dr = float(np.abs(g["disp_r"] - r["disp_r"]).max())
        assert e_dr <= DISP_TOL, f"{label}: random displacement {e_dr}"
    if "delta" in g:
        e_d = rel_l2(g["delta"], r["delta_s"])
        assert e_d <= PSI_TOL, f"{label}: delta rel L2 {e_d}"
    ge, re_ = np.array(g["eps"]), np.array(r["eps"])
    assert ge.shape == re_.shape
    np.testing.assert_allclose(ge, re_, rtol=1e-4, atol=1e-6)


# ---------------------------------------------------------------------------
# Deposit
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("binned", [False, True])
@pytest.mark.parametrize("n", [8, 32, 128])
def test_paint_bitexact_with_weights_wrap_and_order(gpu_lib, n, binned):
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(100 + n)
    box = 300.0
    m = 40000
    pos = (rng.random((m, 3)) * 1.4 * box - 0.2 * box).astype(np.float32)
    pos[:5] = [[0, 0, 0], [box, box, box], [-1e-3, 0, 0], [box * 0.5, 0, box - 1e-4], [1e-7, 1e-7, 1e-7]]
    w = (rng.random(m) * 10).astype(np.float32)
    w[:3] = [0.0, np.float32(2.0 ** -40), np.float32(63.999)]
    plan = native.Plan(n, box, (-100.0, 0.0, 0.0), 1.0, 0.5, 10.0, randoms=True, max_objects=m if binned else 0)
    plan.paint(native.GAL, to_dev(pos), to_dev(w))
    perm = rng.permutation(m)
    plan.paint(native.RAN, to_dev(pos[perm]), to_dev(w[perm]))
    gg = plan.grid(native.GAL)[0].cpu().numpy()
    gr = plan.grid(native.RAN)[0].cpu().numpy()
    ref = O.paint(pos, w, n, box, (0.0, 0.0, 0.0))
    assert np.array_equal(gg, ref)
    assert np.array_equal(gr, ref)
    assert int(gg.sum()) == int(O.quantise_weights(w, m).sum())
    plan.close()


@pytest.mark.parametrize("binned", [False, True])
def test_paint_accumulate_equals_single_call(gpu_lib, binned):
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(7)
    pos = (rng.random((10000, 3)) * 100).astype(np.float32)
    plan = native.Plan(16, 100.0, (50.0, 50.0, 50.0), 1.0, 0.5, 10.0, randoms=False,
                       max_objects=8000 if binned else 0)
    plan.paint(native.GAL, to_dev(pos[:3000]))
    plan.paint(native.GAL, to_dev(pos[3000:]), accumulate=True)
    g = plan.grid(native.GAL)[0].cpu().numpy()
    assert np.array_equal(g, O.paint(pos, None, 16, 100.0, (0, 0, 0)))
    plan.close()


@pytest.mark.parametrize("binned", [False, True])
def test_unit_weight_shares_bitexact(gpu_lib, binned):
    # unit weights take the FP64 share path (floor(c / 2^16), c <= 2^48); objects exactly on nodes
    # (c = 2^48 at corner 0), at cell mid-points and just past a node, with and without a weight array
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(31)
    n = 64
    box = float(n)                                   # cell size 1: integer positions sit on nodes
    m = 60000
    pos = (rng.random((m, 3)) * box).astype(np.float32)
    k = rng.integers(0, n, (3000, 3)).astype(np.float32)
    pos[:1000] = k[:1000]
    pos[1000:2000] = k[1000:2000] + 0.5
    pos[2000:3000] = k[2000:3000] + np.float32(2.0 ** -17)
    ref = O.paint(pos, None, n, box, (0.0, 0.0, 0.0))
    plan = native.Plan(n, box, (-100.0, 0.0, 0.0), 1.0, 0.5, 10.0, randoms=False, max_objects=m if binned else 0)
    plan.paint(native.GAL, to_dev(pos))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), ref)
    plan.paint(native.GAL, to_dev(pos), to_dev(np.ones(m, np.float32)))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), ref)
    plan.close()


def test_sparse_grid_fresh_accumulate_and_densify(gpu_lib):
    # brick-sparse grids: a new deposit clears only the 16^3 bricks it touches, so bricks holding an
    # earlier catalogue must read as zero; an accumulating deposit clears the bricks it adds; an
    # accumulating NGP deposit first makes the grid dense
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(41)
    n, box = 64, 640.0                               # 4 x 4 x 4 bricks of 160 Mpc/h
    full = (rng.random((50000, 3)) * box).astype(np.float32)
    clump = (rng.random((20000, 3)) * 60.0 + 200.0).astype(np.float32)
    edge = (rng.random((5000, 3)) * 8.0 + 472.0).astype(np.float32)    # up to cell 47: footprint into the next brick
    other = (rng.random((3000, 3)) * box).astype(np.float32)
    w = (rng.random(5000) * 3).astype(np.float32)
    plan = native.Plan(n, box, (0.0, 0.0, 0.0), 1.0, 0.5, 10.0, randoms=False, max_objects=50000)
    plan.paint(native.GAL, to_dev(full))
    plan.paint(native.GAL, to_dev(clump))
    ref = O.paint(clump, None, n, box, (0, 0, 0))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), ref)
    plan.paint(native.GAL, to_dev(edge), to_dev(w), accumulate=True)
    ref = ref + O.paint(edge, w, n, box, (0, 0, 0))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), ref)
    plan.paint(native.GAL, to_dev(other), accumulate=True, ngp=True)
    ref = ref + O.paint_ngp(other, None, n, box, (0, 0, 0))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), ref)
    plan.paint(native.GAL, to_dev(clump), accumulate=True)
    ref = ref + O.paint(clump, None, n, box, (0, 0, 0))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), ref)
    plan.close()


def test_sparse_grids_batched_accumulate_and_shift(gpu_lib):
    # batch of 2 with ragged offsets: box-wide catalogues first, then clumps in different bricks per
    # realisation painted anew, then a weighted accumulating deposit; every realisation's grid bit for
    # bit, and the brick-order shift of the catalogue painted last equal to the direct shift
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(47)
    n, box = 64, 640.0
    full = [(rng.random((20000, 3)) * box).astype(np.float32) for _ in range(2)]
    clumps = [(rng.random((7000, 3)) * 50.0 + 100.0).astype(np.float32),
              (rng.random((3000, 3)) * 70.0 + 400.0).astype(np.float32)]
    extra = [(rng.random((500, 3)) * 20.0 + 300.0).astype(np.float32),
             (rng.random((900, 3)) * 20.0 + 150.0).astype(np.float32)]
    w_extra = [(rng.random(e.shape[0]) * 4).astype(np.float32) for e in extra]

    def cat(parts):
        return to_dev(np.concatenate(parts)), to_dev(np.cumsum([0] + [p.shape[0] for p in parts]).astype(np.int64))

    plan = native.Plan(n, box, (320.0, 320.0, 320.0), 1.0, 0.5, 10.0, batch=2, randoms=False, max_objects=40000)
    pos, off = cat(full)
    plan.paint(native.GAL, pos, offsets=off)
    pos, off = cat(clumps)
    plan.paint(native.GAL, pos, offsets=off)
    epos, eoff = cat(extra)
    plan.paint(native.GAL, epos, to_dev(np.concatenate(w_extra)), offsets=eoff, accumulate=True)
    grids = plan.grid(native.GAL).cpu().numpy()
    for i in range(2):
        ref = O.paint(clumps[i], None, n, box, (0, 0, 0)) + O.paint(extra[i], w_extra[i], n, box, (0, 0, 0))
        assert np.array_equal(grids[i], ref), f"realisation {i}"
    plan.solve()
    plan.iterate(2, 0.0)
    d_sorted = plan.shift(native.GAL, epos, offsets=eoff)
    d_direct = plan.shift(native.GAL, epos.clone(), offsets=eoff.clone())
    plan.close()
    assert torch.equal(d_sorted, d_direct)


def test_sparse_grids_after_dense_paint_reconstruct(gpu_lib):
    # grids first filled everywhere by a box-wide catalogue, then the survey catalogues painted anew:
    # the transforms, totals and mask must see only the bricks the survey deposit touched
    from paper_1504_02591_amd import native
    cat = G.config2(n=64, scale=0.125)
    rng = np.random.default_rng(43)
    junk = to_dev((rng.random((cat.ran_pos.shape[0], 3)) * cat.box_len + np.asarray(cat.origin)).astype(np.float32))
    plan = native.plan_for(cat, keep_delta=True)
    plan.paint(native.GAL, junk)
    plan.paint(native.RAN, junk)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve()
    rc, iters, eps = plan.iterate(3, 0.0)
    g = dict(eps=eps[0], psi=plan.psi()[0].cpu().numpy(), grid_g=plan.grid(native.GAL)[0].cpu().numpy(),
             grid_r=plan.grid(native.RAN)[0].cpu().numpy(), disp_g=plan.shift(native.GAL, gal).cpu().numpy(),
             disp_r=plan.shift(native.RAN, ran).cpu().numpy(), delta=plan.delta()[0].cpu().numpy())
    plan.close()
    compare_full(g, oracle_catalogue_run(cat, 3), "sparse grids after a dense paint")


def test_binned_deposit_clustered_and_invalid(gpu_lib):
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(9)
    n, box = 64, 640.0
    pos = np.concatenate([(rng.random((200000, 3)) * 25.0 + 100.0),          # one dense clump
                          rng.random((50000, 3)) * box]).astype(np.float32)
    w = (rng.random(pos.shape[0]) * 3).astype(np.float32)
    plan = native.Plan(n, box, (0.0, 0.0, 0.0), 1.0, 0.5, 10.0, randoms=False, max_objects=pos.shape[0])
    plan.paint(native.GAL, to_dev(pos), to_dev(w))
    assert np.array_equal(plan.grid(native.GAL)[0].cpu().numpy(), O.paint(pos, w, n, box, (0, 0, 0)))
    bad = pos.copy()
    bad[5] = np.inf
    plan.paint(native.GAL, to_dev(bad), to_dev(w))
    with pytest.raises(native.ReconError) as ei:
        plan.solve()
    assert ei.value.code == native.RECON_EINVAL
    plan.close()


# ---------------------------------------------------------------------------
# Transforms and the iteration, fed through the delta hook
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_plane_wave_displacement_gpu(gpu_lib, n):
    from paper_1504_02591_amd import native
    box, amp, ph, b = 400.0, 0.3, 0.7, 1.7
    for modes in [(1, 0, 0), (0, 1, 2), (n // 2 - 1, -2, 1), (3, -1, n // 2 - 1)]:
        delta, k0 = G.plane_wave(n, box, modes, amp, ph)
        plan = native.Plan(n, box, (-1e4, 0, 0), b, 0.0, 0.0, randoms=False)
        plan.set_delta(to_dev(delta.astype(np.float32)))
        plan.solve()
        plan.iterate(1, 0.0)
        psi = plan.psi()[0].cpu().numpy()
        plan.close()
        h = box / n
        i = np.arange(n) * h
        z, y, x = np.meshgrid(i, i, i, indexing="ij")
        arg = k0[0] * x + k0[1] * y + k0[2] * z + ph
        expect = np.stack([-(amp / (b * float(k0 @ k0))) * k0[j] * np.sin(arg) for j in range(3)])
        assert rel_l2(psi, expect) < PSI_TOL, modes


@pytest.mark.parametrize("n,observer", [(8, (31.3, 47.9, 52.1)), (16, (-80.0, 130.0, 60.0)),
                                        (32, (150.0, 150.0, 150.0)), (64, (-300.0, 100.0, 250.0)),
                                        (128, (200.0, 200.0, 200.0)), (256, (-50.0, 210.0, 190.0))])
def test_random_field_iterates_match_oracle(gpu_lib, n, observer):
    from paper_1504_02591_amd import native
    box, b, f = 400.0, 1.5, 0.6
    rng = np.random.default_rng(200 + n)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 2.5 * box / n)
    for npass in (1, 3):
        plan = native.Plan(n, box, observer, b, f, 0.0, randoms=False)
        plan.set_delta(to_dev(delta.astype(np.float32)))
        plan.solve()
        rc, iters, eps = plan.iterate(npass, 0.0)
        psi = plan.psi()[0].cpu().numpy()
        plan.close()
        ref = O.reconstruct_field(delta.astype(np.float32).astype(np.float64), box, (0, 0, 0), observer, b, f,
                                  n_passes=npass)
        e = rel_l2(psi, ref["psi"])
        print(f"n={n} passes={npass} relL2={e:.2e}", flush=True)
        assert iters[0] == npass
        assert e < PSI_TOL
        np.testing.assert_allclose(eps[0], ref["eps"], rtol=1e-4, atol=1e-6)


def test_full_size_pass_matches_oracle(gpu_lib):
    """512^3, the benchmarked launch configuration: two passes from a survey-like field vs the oracle."""
    from paper_1504_02591_amd import native
    n, box, b, f = 512, 3500.0, 2.0, 0.74
    obs = (1750.0, 1750.0, 1750.0)
    delta, _ = G.linear_field(n, box, 77, want_psi=False, dtype=np.float32)
    delta = delta.astype(np.float32)
    plan = native.Plan(n, box, obs, b, f, 15.0, randoms=False)
    plan.set_delta(to_dev(delta))
    plan.solve()
    rc, iters, eps = plan.iterate(2, 0.0)
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    ref = O.reconstruct_field(delta.astype(np.float64), box, (0, 0, 0), obs, b, f, n_passes=2)
    e = rel_l2(psi, ref["psi"])
    print(f"512^3 two passes: psi relL2={e:.2e} eps gpu={eps[0]} oracle={ref['eps']}", flush=True)
    assert e < PSI_TOL
    np.testing.assert_allclose(eps[0], ref["eps"], rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("axis", [0, 2])
def test_distant_observer_closed_form_gpu(gpu_lib, axis):
    from paper_1504_02591_amd import native
    n, box, b, f = 32, 400.0, 2.0, 0.74
    beta = f / b
    rng = np.random.default_rng(31 + axis)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 30.0).astype(np.float32)
    obs = [box / 2] * 3
    obs[axis] -= 1e9 * box
    plan = native.Plan(n, box, obs, b, f, 0.0, randoms=False)
    plan.set_delta(to_dev(delta))
    plan.solve()
    plan.iterate(4, 0.0)
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    d = delta.astype(np.float64)
    m = np.fft.fftfreq(n, d=1.0 / n)
    kk = [(2 * np.pi / box) * m.reshape(1, 1, -1), (2 * np.pi / box) * m.reshape(1, -1, 1),
          (2 * np.pi / box) * m.reshape(-1, 1, 1)]
    mm = [m.reshape(1, 1, -1), m.reshape(1, -1, 1), m.reshape(-1, 1, 1)]
    dk = [np.where(np.abs(a) == n // 2, 0.0, k) for a, k in zip(mm, kk)]
    k2 = kk[0] ** 2 + kk[1] ** 2 + kk[2] ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        mu2 = np.where(k2 > 0, dk[axis] ** 2 / k2, 0.0)
        dn = np.fft.fftn(d) * (1 - (-beta * mu2) ** 5) / (1 + beta * mu2)
        pot = np.where(k2 > 0, dn / (b * k2), 0.0)
    expect = np.stack([np.real(np.fft.ifftn(1j * dk[j] * pot)) for j in range(3)])
    assert rel_l2(psi, expect) < PSI_TOL


# ---------------------------------------------------------------------------
# End to end on catalogues
# ---------------------------------------------------------------------------
def test_config1_end_to_end(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.config1()
    g = gpu_catalogue_run(native, cat, 6)
    r = oracle_catalogue_run(cat, 6)
    compare_full(g, r, "config1")


def test_precision_study_subrun(gpu_lib):
    # the precision-study geometry (L = 2000, f = 0.76, b = 1, distant observer 5000 Mpc/h from the
    # centre, lattice of Zel'dovich particles, no randoms) on its 128^3 sub-run: FP32 GPU vs FP64 oracle
    from paper_1504_02591_amd import native
    cat = G.config3(128)
    g = gpu_catalogue_run(native, cat, 6)
    r = oracle_catalogue_run(cat, 6)
    e = rel_l2(g["psi"], r["psi"])
    print(f"precision study 128^3: Psi rel L2 (FP32 GPU vs FP64 oracle) = {e:.3e}", flush=True)
    compare_full(g, r, "precision-study 128^3")


@pytest.mark.parametrize("terms", [2, 3])
def test_precision_study_split_bf16_radix(gpu_lib, terms):
    # the same sub-run with the last radix-8 stage of the steady passes' z transforms on the matrix
    # cores (8-point DFT as a GEMM on split-bfloat16 operands): the grid and the first pass are the
    # FP32 path's; the error against the FP64 oracle is reported.  Three terms keep FP32-level error;
    # two terms (about 2^-16 per product) are held to a looser bar
    from paper_1504_02591_amd import native
    cat = G.config3(128)
    plan = native.plan_for(cat, split_terms=terms)
    gal = to_dev(cat.gal_pos)
    plan.paint(native.GAL, gal)
    plan.solve()
    rc, iters, eps = plan.iterate(6, 0.0)
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    r = oracle_catalogue_run(cat, 6)
    e = rel_l2(psi, r["psi"])
    print(f"precision study 128^3, split-bf16 radix ({terms} terms): Psi rel L2 vs FP64 oracle = {e:.3e}; "
          f"eps {eps[0]}", flush=True)
    assert e <= (PSI_TOL if terms == 3 else 1e-3)
    np.testing.assert_allclose(eps[0], r["eps"], rtol=1e-2 if terms == 2 else 1e-4, atol=1e-6)


def test_survey_cone_small(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.config2(n=128, scale=0.25)
    g = gpu_catalogue_run(native, cat, 5)
    r = oracle_catalogue_run(cat, 5)
    compare_full(g, r, "survey128")


def test_mean_density_mode(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.config3(n=64)
    g = gpu_catalogue_run(native, cat, 4)
    r = oracle_catalogue_run(cat, 4)
    compare_full(g, r, "meandensity64")


@pytest.mark.parametrize("start", [1, 2])
def test_ffta_starts(gpu_lib, start):
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 21, 22, ran_factor=3, bias=1.2, smooth_r=20.0)
    for npass in (1, 2, 4):
        g = gpu_catalogue_run(native, cat, npass, start=start)
        r = oracle_catalogue_run(cat, npass, start=start)
        compare_full(g, r, f"ffta{start}-{npass}")


@pytest.mark.parametrize("survey", [False, True, "cone"])
def test_lognormal_option_matches_oracle(gpu_lib, survey):
    # Sec. 6, eq. (logdelta): kept field, Psi, eps and shifts against the oracle's transform; the cone
    # case has z tiles wholly outside the survey mask (no transform, zero log-mean partials)
    from paper_1504_02591_amd import native
    if survey == "cone":
        cat = G.config2(n=64, scale=0.125)
    elif survey:
        cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 25, 26, ran_factor=3, bias=1.2, smooth_r=20.0)
    else:
        cat = G.config3(32)
    g = gpu_catalogue_run(native, cat, 3, lognormal=True)
    r = oracle_catalogue_run(cat, 3, log_transform=True)
    compare_full(g, r, f"lognormal survey={survey}")


@pytest.mark.parametrize("n", [16, 64])
def test_ngp_deposit_bitexact(gpu_lib, n):
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(40 + n)
    box = 300.0
    m = 20000
    pos = (rng.random((m, 3)) * 1.2 * box - 0.1 * box).astype(np.float32)
    pos[:3] = np.array([[0.0, 0.0, 0.0], [box / n * 0.5, box / n * 1.5, box - 1e-3], [-box / n * 0.5, 3.0, 7.0]],
                       dtype=np.float32)
    w = (rng.random(m) * 5).astype(np.float32)
    plan = native.Plan(n, box, (0.0, 0.0, -1000.0), 1.0, 0.5, 10.0, randoms=False)
    plan.paint(native.GAL, to_dev(pos), to_dev(w), ngp=True)
    grid = plan.grid(native.GAL)[0].cpu().numpy()
    plan.close()
    assert np.array_equal(grid, O.paint_ngp(pos, w, n, box, (0.0, 0.0, 0.0)))


def test_ngp_deposit_batched_ragged(gpu_lib):
    """The NGP deposit over a batch of three realisations with ragged offsets (the middle one empty,
    the others of different sizes, weighted): each realisation's grid bit for bit, the empty one all
    zeros."""
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(77)
    n, box = 32, 320.0
    parts = [(rng.random((5000, 3)) * box).astype(np.float32), np.zeros((0, 3), np.float32),
             (rng.random((1700, 3)) * 80.0 + 100.0).astype(np.float32)]
    ws = [(rng.random(p.shape[0]) * 3).astype(np.float32) for p in parts]
    pos, w = np.concatenate(parts), np.concatenate(ws)
    off = np.cumsum([0] + [p.shape[0] for p in parts]).astype(np.int64)
    plan = native.Plan(n, box, (160.0, 160.0, 160.0), 1.0, 0.5, 10.0, batch=3, randoms=False)
    plan.paint(native.GAL, to_dev(pos), to_dev(w), offsets=to_dev(off), ngp=True)
    grids = plan.grid(native.GAL).cpu().numpy()
    plan.close()
    for i, (p, wi) in enumerate(zip(parts, ws)):
        assert np.array_equal(grids[i], O.paint_ngp(p, wi, n, box, (0.0, 0.0, 0.0))), f"realisation {i}"
    assert not grids[1].any() and grids[0].any() and grids[2].any()


def test_ngp_reconstruction_matches_oracle(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 27, 28, ran_factor=3, bias=1.2, smooth_r=20.0)
    plan = native.plan_for(cat, keep_delta=True)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal, ngp=True)
    plan.paint(native.RAN, ran, ngp=True)
    plan.solve()
    rc, iters, eps = plan.iterate(3, 0.0)
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    gg = O.paint_ngp(cat.gal_pos, None, cat.n, cat.box_len, cat.origin)
    gr = O.paint_ngp(cat.ran_pos, None, cat.n, cat.box_len, cat.origin)
    delta = O.overdensity(gg, gr, cat.box_len, cat.smooth_r, cat.mask_tau)
    ref = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth, n_passes=3)
    assert rel_l2(psi, ref["psi"]) < PSI_TOL
    np.testing.assert_allclose(eps[0], ref["eps"], rtol=1e-4, atol=1e-6)


def test_radial_ratio_statistic_matches_oracle(gpu_lib):
    # Sec. 4 Table 1 statistic: the lattice's true linear displacement against Psi after one pass
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 29, 30, ran_factor=3, bias=1.0, smooth_r=20.0)
    _, psi_true = G.linear_field(cat.n, cat.box_len, cat.info["seed_field"])
    plan = native.plan_for(cat)
    plan.paint(native.GAL, to_dev(cat.gal_pos))
    plan.paint(native.RAN, to_dev(cat.ran_pos))
    plan.solve()
    plan.iterate(1, 0.0)
    stats = plan.radial_ratio(to_dev(np.ascontiguousarray(psi_true[None], dtype=np.float32)))[0]
    plan.close()
    r = oracle_catalogue_run(cat, 1)
    rhat = O.line_of_sight(cat.n, cat.box_len, cat.origin, cat.observer)
    ref = O.radial_ratio_stats(psi_true, r["psi"], rhat)
    print(f"radial ratio gpu {stats} oracle {ref}", flush=True)
    assert abs(stats[0] - ref[0]) < 1e-4 and abs(stats[1] - ref[1]) < 1e-4
    assert abs(stats[3] - ref[3]) <= 2 and abs(stats[2] - ref[2]) <= 2.0 / cat.n ** 3


@pytest.mark.parametrize("n", [16, 64])
def test_helmholtz_split_matches_oracle(gpu_lib, n):
    # Sec. 4.1: irrotational and solenoidal parts of (Psi.x) x for the x displacement of a linear field
    from paper_1504_02591_amd import native
    box = 8.0 * n
    _, psi = G.linear_field(n, box, 90 + n)
    px = np.ascontiguousarray(psi[0], dtype=np.float32)
    plan = native.Plan(n, box, (0.0, 0.0, -5 * box), 1.7, 0.6, 0.0, randoms=False, batch=2)
    irr, sol = plan.helmholtz(to_dev(np.stack([px, 2.0 * px])))
    irr, sol = irr.cpu().numpy(), sol.cpu().numpy()
    with pytest.raises(native.ReconError):
        plan.psi()                      # the plan was reset
    plan.close()
    ri, rs = O.helmholtz_x(px.astype(np.float64), box)
    for b, fac in ((0, 1.0), (1, 2.0)):
        assert rel_l2(irr[b], fac * ri) < PSI_TOL
        assert rel_l2(sol[b], fac * rs) < PSI_TOL


def test_batched_matches_single_realisations(gpu_lib):
    from paper_1504_02591_amd import native
    cats = [G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 30 + i, 40 + i, ran_factor=2, bias=1.0,
                          smooth_r=20.0, n_part=24 + 4 * i) for i in range(3)]
    gal = np.concatenate([c.gal_pos for c in cats])
    ran = np.concatenate([c.ran_pos for c in cats])
    goff = np.cumsum([0] + [c.gal_pos.shape[0] for c in cats]).astype(np.int64)
    roff = np.cumsum([0] + [c.ran_pos.shape[0] for c in cats]).astype(np.int64)
    c0 = cats[0]
    plan = native.Plan(32, 500.0, c0.observer, 1.0, 0.7, 20.0, batch=3, max_objects=ran.shape[0])
    plan.paint(native.GAL, to_dev(gal), offsets=to_dev(goff))
    plan.paint(native.RAN, to_dev(ran), offsets=to_dev(roff))
    plan.solve()
    rc, iters, eps = plan.iterate(3, 0.0)
    psi = plan.psi().cpu().numpy()
    disp = plan.shift(native.GAL, to_dev(gal), offsets=to_dev(goff)).cpu().numpy()
    grids = plan.grid(native.GAL).cpu().numpy()
    plan.close()
    for i, c in enumerate(cats):
        r = oracle_catalogue_run(c, 3)
        assert np.array_equal(grids[i], r["grid_g"])
        assert rel_l2(psi[i], r["psi"]) < PSI_TOL
        assert np.abs(disp[goff[i]:goff[i + 1]] - r["disp_g"]).max() < DISP_TOL
        np.testing.assert_allclose(eps[i], r["eps"], rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("last", ["gal", "ran"])
def test_shift_in_brick_order_equals_direct_shift(gpu_lib, last, n):
    # the shift of the catalogue painted last (same buffer, count and offsets) runs on the deposit's
    # brick-ordered copy and is put back in input order; a copy of the positions in another buffer takes
    # the direct path.  Both must agree bit for bit (galaxies with the RSD term, randoms without), with
    # the shifted positions, and with the oracle
    from paper_1504_02591_amd import native
    # n = 8 and 16: one 16^3 brick covers the whole grid and its footprint wraps onto itself
    cat = G.lattice_box(n, 500.0, (-500.0, 250.0, 250.0), 0.7, 21, 22, ran_factor=3, bias=1.2, smooth_r=20.0)
    plan = native.plan_for(cat)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    order = [(native.RAN, ran), (native.GAL, gal)] if last == "gal" else [(native.GAL, gal), (native.RAN, ran)]
    for which, pos in order:
        plan.paint(which, pos)
    plan.solve()
    plan.iterate(3, 0.0)
    which, pos = order[-1]
    d_sorted, p_sorted = plan.shift(which, pos, want_pos=True)
    d_direct, p_direct = plan.shift(which, pos.clone(), want_pos=True)
    plan.close()
    diff = (d_sorted != d_direct).any(dim=1)
    if bool(diff.any()):
        idx = torch.nonzero(diff).flatten()[:5].cpu().numpy()
        r = oracle_catalogue_run(cat, 3)
        ref = r["disp_g"] if which == native.GAL else r["disp_r"]
        print(f"{int(diff.sum())} of {diff.numel()} differ; max |d| {float((d_sorted - d_direct).abs().max()):.3e}; "
              f"sorted vs oracle {float(np.abs(d_sorted.cpu().numpy() - ref).max()):.3e}, direct vs oracle "
              f"{float(np.abs(d_direct.cpu().numpy() - ref).max()):.3e}; first {idx} pos {pos[idx].cpu().numpy()} "
              f"sorted {d_sorted[idx].cpu().numpy()} direct {d_direct[idx].cpu().numpy()}", flush=True)
    assert torch.equal(d_sorted, d_direct)
    assert torch.equal(p_sorted, p_direct)
    assert torch.equal(p_sorted, pos + d_sorted)     # the shifted position is fl32(x + d)
    r = oracle_catalogue_run(cat, 3)
    ref = r["disp_g"] if which == native.GAL else r["disp_r"]
    assert float(np.abs(d_sorted.cpu().numpy() - ref).max()) <= DISP_TOL


def test_brick_order_shift_needs_the_unchanged_painted_catalogue(gpu_lib):
    # the deposit's brick-ordered copy stands in for the positions only when the caller passes the very
    # tensor painted last, unchanged: another catalogue of the same length (whatever its address) and
    # the painted tensor changed in place both take the direct path; at the C ABI a false claim of
    # RECON_SHIFT_AS_PAINTED is refused
    import ctypes
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 41, 42, ran_factor=3, bias=1.2, smooth_r=20.0)
    plan = native.plan_for(cat)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve()
    plan.iterate(2, 0.0)
    del ran                                            # the plan still holds the painted tensor
    other = to_dev((cat.ran_pos[::-1] * np.float32(0.97)).copy())
    d_other = plan.shift(native.RAN, other)
    d_other_direct = plan.shift(native.RAN, other.clone())
    assert torch.equal(d_other, d_other_direct)
    painted = plan._painted[1]
    painted.mul_(0.99)                                 # changed in place after the paint
    d_changed = plan.shift(native.RAN, painted)
    d_changed_direct = plan.shift(native.RAN, painted.clone())
    assert torch.equal(d_changed, d_changed_direct)
    disp = torch.empty_like(other)
    rc = plan.lib.recon_shift(plan.handle, native.RAN | native.SHIFT_AS_PAINTED, ctypes.c_void_p(other.data_ptr()),
                              other.shape[0], None, ctypes.c_void_p(disp.data_ptr()), None)
    assert rc == native.RECON_EINVAL
    plan.close()
    r = O.reconstruct(cat.gal_pos, None, cat.ran_pos, None, cat.n, cat.box_len, cat.origin, cat.observer,
                      cat.bias, cat.growth, cat.smooth_r, cat.mask_tau, n_passes=2)
    ref = O.shift(r["psi"], other.cpu().numpy(), cat.box_len, cat.origin, cat.observer, cat.growth, False)
    assert np.abs(d_other.cpu().numpy() - ref).max() <= DISP_TOL


def test_shift_in_brick_order_batched(gpu_lib):
    from paper_1504_02591_amd import native
    cats = [G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 50 + i, 60 + i, ran_factor=2, bias=1.0,
                          smooth_r=20.0, n_part=24 + 4 * i) for i in range(3)]
    gal = to_dev(np.concatenate([c.gal_pos for c in cats]))
    ran = to_dev(np.concatenate([c.ran_pos for c in cats]))
    goff = to_dev(np.cumsum([0] + [c.gal_pos.shape[0] for c in cats]).astype(np.int64))
    roff_np = np.cumsum([0] + [c.ran_pos.shape[0] for c in cats]).astype(np.int64)
    roff = to_dev(roff_np)
    c0 = cats[0]
    plan = native.Plan(32, 500.0, c0.observer, 1.0, 0.7, 20.0, batch=3, max_objects=int(ran.shape[0]))
    plan.paint(native.GAL, gal, offsets=goff)
    plan.paint(native.RAN, ran, offsets=roff)
    plan.solve()
    plan.iterate(3, 0.0)
    d_sorted = plan.shift(native.RAN, ran, offsets=roff)
    d_direct = plan.shift(native.RAN, ran.clone(), offsets=roff.clone())
    plan.close()
    assert torch.equal(d_sorted, d_direct)
    d = d_sorted.cpu().numpy()
    for i, c in enumerate(cats):
        r = oracle_catalogue_run(c, 3)
        assert np.abs(d[roff_np[i]:roff_np[i + 1]] - r["disp_r"]).max() < DISP_TOL


# ---------------------------------------------------------------------------
# Tolerance mode, divergence and errors
# ---------------------------------------------------------------------------
def test_tolerance_mode_counts_passes(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.5, 51, 52, ran_factor=2, bias=1.0, smooth_r=20.0)
    g = gpu_catalogue_run(native, cat, 40, tol=1e-3)
    r = O.reconstruct(cat.gal_pos, None, cat.ran_pos, None, cat.n, cat.box_len, cat.origin, cat.observer,
                      cat.bias, cat.growth, cat.smooth_r, cat.mask_tau, tol=1e-3, max_iter=40)
    assert g["rc"] == 0
    assert abs(g["iters"] - r["passes"]) <= 1
    assert g["eps"][-1] <= 1e-3


@pytest.mark.parametrize("stop_at", [1, 2])
def test_start_tolerance_stop_returns_that_pass(gpu_lib, stop_at):
    # eps_1 of an FFTA start is only known during the next pass: stopping at pass 1 must still
    # return Psi_1, and stopping at pass 2 Psi_2
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 61, 62, ran_factor=3, bias=1.2, smooth_r=20.0)
    ref3 = oracle_catalogue_run(cat, 3, start=native.START_FFTA2)
    e = ref3["eps"]
    assert e[0] > e[1] > e[2]
    tol = e[stop_at - 1] * 1.01
    g = gpu_catalogue_run(native, cat, 10, start=native.START_FFTA2, tol=tol)
    r = oracle_catalogue_run(cat, stop_at, start=native.START_FFTA2)
    assert g["rc"] == 0 and g["iters"] == stop_at
    assert len(g["eps"]) == stop_at
    compare_full(g, r, f"ffta2 stop at {stop_at}")


@pytest.mark.parametrize("batch", [1, 2])
def test_pass_graph_replays_match_eager(gpu_lib, batch):
    # the captured steady-state pass, replayed with eager work and synchronisation in between,
    # must reproduce the eager passes bit for bit
    from paper_1504_02591_amd import native
    n, box = 32, 400.0
    rng = np.random.default_rng(12)
    delta = np.stack([O.smooth(rng.standard_normal((n, n, n)), box, 25.0) for _ in range(batch)]).astype(np.float32)
    runs = []
    for graphs in (False, True):
        plan = native.Plan(n, box, (30.0, -50.0, 400.0), 1.5, 0.8, 0.0, randoms=False, batch=batch, graphs=graphs)
        plan.set_delta(to_dev(delta))
        plan.solve()
        out = []
        for _ in range(3):
            rc, iters, eps = plan.iterate(2, 0.0)
            psi = plan.psi().cpu().numpy()
            torch.cuda.synchronize()
            out.append((list(iters), [list(e) for e in eps], psi))
        plan.close()
        runs.append(out)
    for (ie, ee, pe), (ig, eg, pg) in zip(*runs):
        assert ie == ig and ee == eg
        assert np.array_equal(pe, pg)


def test_fixed_passes_past_convergence_do_not_diverge(gpu_lib):
    # FP32 eps settles at its rounding floor and may rise there; that must not read as divergence
    from paper_1504_02591_amd import native
    n, box = 32, 400.0
    rng = np.random.default_rng(13)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 25.0).astype(np.float32)
    plan = native.Plan(n, box, (200.0, 200.0, -1200.0), 2.0, 0.74, 0.0, randoms=False)
    plan.set_delta(to_dev(delta))
    plan.solve()
    rc, iters, eps = plan.iterate(40, 0.0)
    plan.close()
    assert rc == native.RECON_OK and iters[0] == 40
    assert min(eps[0]) < 1e-5


def test_not_converged_and_resume(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 53, 54, ran_factor=2, bias=1.0, smooth_r=20.0)
    plan = native.plan_for(cat)
    plan.paint(native.GAL, to_dev(cat.gal_pos))
    plan.paint(native.RAN, to_dev(cat.ran_pos))
    plan.solve()
    rc, iters, eps = plan.iterate(2, 1e-9)
    assert rc == native.RECON_NOTCONVERGED and iters[0] == 2
    rc, iters, eps = plan.iterate(2, 1e-9)
    assert iters[0] == 4
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    r = oracle_catalogue_run(cat, 4)
    assert rel_l2(psi, r["psi"]) < PSI_TOL


@pytest.mark.parametrize("start", [0, 2])
@pytest.mark.parametrize("graphs", [False, True])
def test_split_iterate_calls_equal_one_call(gpu_lib, start, graphs):
    # a call ends on the full fan-out (Psi written); the next call turns it into the iteration's
    # combined form, or rebuilds state X when none is left: the passes must be the same bit for bit
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 55, 56, ran_factor=2, bias=1.1, smooth_r=20.0)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    out = []
    for split in ((5,), (0, 2, 3)):
        plan = native.plan_for(cat, start_buffers=start != 0, graphs=graphs)
        plan.paint(native.GAL, gal)
        plan.paint(native.RAN, ran)
        plan.solve(start)
        eps = []
        for k in split:
            rc, iters, e = plan.iterate(k, 0.0)
            eps += list(e[0])
        out.append((iters[0], eps, plan.psi()[0].cpu().numpy()))
        plan.close()
    (i1, e1, p1), (i2, e2, p2) = out
    assert i1 == i2 == 5
    assert e1 == e2
    assert np.array_equal(p1, p2)


def test_divergence_detected(gpu_lib):
    from paper_1504_02591_amd import native
    n, box = 16, 300.0
    rng = np.random.default_rng(3)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 30.0).astype(np.float32)
    plan = native.Plan(n, box, (150.0, 150.0, -3e9), 1.0, 2.5, 0.0, randoms=False)
    plan.set_delta(to_dev(delta))
    plan.solve()
    with pytest.raises(native.ReconError) as ei:
        plan.iterate(30, 1e-6)
    assert ei.value.code == native.RECON_EDIVERGED
    plan.close()


@pytest.mark.parametrize("start", ["plain", "ffta2"])
def test_nonfinite_field_reads_as_divergence(gpu_lib, start):
    # a non-finite overdensity (e.g. from a broken upstream step) must end in EDIVERGED, not in a
    # clipped convergence norm of 0 that reports a NaN displacement as converged
    from paper_1504_02591_amd import native
    n, box = 16, 300.0
    rng = np.random.default_rng(4)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 30.0).astype(np.float32)
    delta[3, 5, 7] = np.nan
    plan = native.Plan(n, box, (150.0, 150.0, -500.0), 2.0, 0.7, 0.0, randoms=False, start_buffers=True)
    plan.set_delta(to_dev(delta))
    plan.solve(native.START_PLAIN if start == "plain" else native.START_FFTA2)
    with pytest.raises(native.ReconError) as ei:
        plan.iterate(10, 1e-3)
    assert ei.value.code == native.RECON_EDIVERGED
    plan.close()


@pytest.mark.parametrize("mask_tau", [0.0, 0.6])
def test_mask_threshold(gpu_lib, mask_tau):
    """The survey end to end at other mask thresholds (tau = 0: every cell whose 27-cell window holds
    random weight, 37,523 cells at 64^3; 0.6: a tighter footprint, 22,691 cells; the default 0.1 gives
    29,972): grids, mask (through delta), Psi, eps and shifts against the oracle."""
    from paper_1504_02591_amd import native
    cat = G.config2(n=64, scale=0.125)
    plan = native.Plan(cat.n, cat.box_len, cat.observer, cat.bias, cat.growth, cat.smooth_r, origin=cat.origin,
                       mask_tau=mask_tau, max_objects=cat.ran_pos.shape[0], keep_delta=True)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve()
    rc, iters, eps = plan.iterate(3, 0.0)
    tiles = plan.tile_counts()[0]
    g = dict(eps=eps[0], psi=plan.psi()[0].cpu().numpy(), grid_g=plan.grid(native.GAL)[0].cpu().numpy(),
             grid_r=plan.grid(native.RAN)[0].cpu().numpy(), disp_g=plan.shift(native.GAL, gal).cpu().numpy(),
             disp_r=plan.shift(native.RAN, ran).cpu().numpy(), delta=plan.delta()[0].cpu().numpy())
    plan.close()
    r = O.reconstruct(cat.gal_pos, None, cat.ran_pos, None, cat.n, cat.box_len, cat.origin, cat.observer,
                      cat.bias, cat.growth, cat.smooth_r, mask_tau, n_passes=3)
    mask = O.survey_mask(r["grid_r"], mask_tau)
    print(f"tau={mask_tau}: {int(np.count_nonzero(mask))} cells inside the mask, mask tiles {tiles[2]} of "
          f"{tiles[3]}", flush=True)
    tw = cat.n * cat.n // tiles[3]                     # z tile: one y row, tw consecutive x
    assert tiles[2] == int(mask.any(axis=0).reshape(cat.n, -1, tw).any(axis=2).sum())
    compare_full(g, r, f"tau={mask_tau}")


def test_no_smoothing_mean_density(gpu_lib):
    """R = 0 (S(k) = 1) on the Zel'dovich lattice box without randoms (delta = G/rho_bar - 1 straight
    from the CIC grid): grid, delta, Psi, eps and the shift against the oracle."""
    from paper_1504_02591_amd import native
    cat = G.config3(n=64)
    plan = native.Plan(cat.n, cat.box_len, cat.observer, cat.bias, cat.growth, 0.0, origin=cat.origin,
                       randoms=False, max_objects=cat.gal_pos.shape[0], keep_delta=True)
    gal = to_dev(cat.gal_pos)
    plan.paint(native.GAL, gal)
    plan.solve()
    rc, iters, eps = plan.iterate(3, 0.0)
    g = dict(eps=eps[0], psi=plan.psi()[0].cpu().numpy(), grid_g=plan.grid(native.GAL)[0].cpu().numpy(),
             disp_g=plan.shift(native.GAL, gal).cpu().numpy(), delta=plan.delta()[0].cpu().numpy())
    plan.close()
    r = O.reconstruct(cat.gal_pos, None, None, None, cat.n, cat.box_len, cat.origin, cat.observer, cat.bias,
                      cat.growth, 0.0, cat.mask_tau, n_passes=3)
    compare_full(g, r, "R=0, mean density")


def test_box_origin_offset_matches_oracle(gpu_lib):
    """A survey whose box does not start at the coordinate origin: objects, observer and box origin
    moved by one vector (the translated positions rounded to float32 as a caller would hold them).
    Grids bit for bit, Psi, eps and both catalogues' shifts against the oracle on the same inputs, and
    Psi close to the untranslated reconstruction (the rounding of the positions moves a few CIC
    fractions by one 2^-16 step)."""
    from paper_1504_02591_amd import native
    cat = G.config2(n=64, scale=0.125)
    off = np.array([-1000.0, 250.0, 3000.0])
    gal = (cat.gal_pos.astype(np.float64) + off).astype(np.float32)
    ran = (cat.ran_pos.astype(np.float64) + off).astype(np.float32)
    obs = tuple(np.asarray(cat.observer) + off)
    plan = native.Plan(cat.n, cat.box_len, obs, cat.bias, cat.growth, cat.smooth_r, origin=tuple(off),
                       mask_tau=cat.mask_tau, max_objects=ran.shape[0], keep_delta=True)
    g_gal, g_ran = to_dev(gal), to_dev(ran)
    plan.paint(native.GAL, g_gal)
    plan.paint(native.RAN, g_ran)
    plan.solve()
    rc, iters, eps = plan.iterate(3, 0.0)
    g = dict(eps=eps[0], psi=plan.psi()[0].cpu().numpy(), grid_g=plan.grid(native.GAL)[0].cpu().numpy(),
             grid_r=plan.grid(native.RAN)[0].cpu().numpy(), disp_g=plan.shift(native.GAL, g_gal).cpu().numpy(),
             disp_r=plan.shift(native.RAN, g_ran).cpu().numpy(), delta=plan.delta()[0].cpu().numpy())
    plan.close()
    r = O.reconstruct(gal, None, ran, None, cat.n, cat.box_len, tuple(off), obs, cat.bias, cat.growth,
                      cat.smooth_r, cat.mask_tau, n_passes=3)
    compare_full(g, r, "box origin offset")
    base = oracle_catalogue_run(cat, 3)
    e = rel_l2(g["psi"], base["psi"])
    print(f"box origin offset: psi rel L2 against the untranslated reconstruction {e:.2e}", flush=True)
    assert e < 1e-4                 # the oracle alone: 1.3e-6; a wrong sign of the origin gives O(1)


def test_zero_galaxy_weight_is_refused(gpu_lib):
    """A realisation without galaxy weight has no overdensity (alpha = W_g/W_r = 0, or rho_bar = 0
    without randoms; Sec. 2, Sec. 3.2): recon_solve returns EINVAL, as the oracle raises.  An empty
    catalogue, one of zero weights, and an empty realisation inside a batch; the plan then takes a
    valid catalogue and matches the oracle."""
    from paper_1504_02591_amd import native
    rng = np.random.default_rng(11)
    n, box, obs = 16, 160.0, (80.0, 80.0, 80.0)
    gal = (rng.random((150, 3)) * box).astype(np.float32)
    ran = (rng.random((3000, 3)) * box).astype(np.float32)
    empty = to_dev(np.zeros((0, 3), np.float32))

    def refused(plan):
        with pytest.raises(native.ReconError) as ei:
            plan.solve()
        assert ei.value.code == native.RECON_EINVAL and "galaxy weight" in str(ei.value)

    plan = native.Plan(n, box, obs, 1.0, 0.5, 10.0, max_objects=ran.shape[0])
    plan.paint(native.GAL, empty)
    plan.paint(native.RAN, to_dev(ran))
    refused(plan)
    plan.paint(native.GAL, to_dev(gal), to_dev(np.zeros(gal.shape[0], np.float32)))
    plan.paint(native.RAN, to_dev(ran))
    refused(plan)
    plan.paint(native.GAL, to_dev(gal))
    plan.paint(native.RAN, to_dev(ran))
    plan.solve()
    plan.iterate(2, 0.0)
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    r = O.reconstruct(gal, None, ran, None, n, box, (0.0, 0.0, 0.0), obs, 1.0, 0.5, 10.0, 0.1, n_passes=2)
    assert rel_l2(psi, r["psi"]) < PSI_TOL
    with pytest.raises(ValueError, match="galaxy weight"):
        O.reconstruct(gal[:0], None, ran, None, n, box, (0.0, 0.0, 0.0), obs, 1.0, 0.5, 10.0, 0.1, n_passes=2)

    # batch of 2, realisation 0 without galaxies (offsets 0, 0, 150), the binned deposit
    plan = native.Plan(n, box, obs, 1.0, 0.5, 10.0, batch=2, max_objects=2 * ran.shape[0])
    plan.paint(native.GAL, to_dev(gal), offsets=to_dev(np.array([0, 0, gal.shape[0]], np.int64)))
    plan.paint(native.RAN, to_dev(np.concatenate([ran, ran])),
               offsets=to_dev(np.array([0, ran.shape[0], 2 * ran.shape[0]], np.int64)))
    refused(plan)
    plan.close()

    # mean-density mode (no randoms): rho_bar = 0
    plan = native.Plan(n, box, obs, 1.0, 0.5, 10.0, randoms=False)
    plan.paint(native.GAL, empty)
    refused(plan)
    plan.close()


def test_invalid_inputs_and_order(gpu_lib):
    from paper_1504_02591_amd import native
    plan = native.Plan(16, 100.0, (50.0, 50.0, 50.0), 1.0, 0.5, 10.0)
    with pytest.raises(native.ReconError) as ei:
        plan.solve()
    assert ei.value.code == native.RECON_ESTATE
    with pytest.raises(native.ReconError) as ei:
        plan.iterate(1, 0.0)
    assert ei.value.code == native.RECON_ESTATE
    pos = np.random.default_rng(1).random((100, 3)).astype(np.float32) * 100
    bad = pos.copy()
    bad[17, 1] = np.nan
    plan.paint(native.GAL, to_dev(bad))
    plan.paint(native.RAN, to_dev(pos))
    with pytest.raises(native.ReconError) as ei:
        plan.solve()
    assert ei.value.code == native.RECON_EINVAL
    plan.paint(native.GAL, to_dev(pos), to_dev(np.full(100, -1.0, np.float32)))
    plan.paint(native.RAN, to_dev(pos))
    with pytest.raises(native.ReconError) as ei:
        plan.solve()
    assert ei.value.code == native.RECON_EINVAL
    plan.paint(native.GAL, to_dev(pos))
    plan.paint(native.RAN, to_dev(pos), to_dev(np.zeros(100, np.float32)))
    with pytest.raises(native.ReconError) as ei:
        plan.solve()
    assert ei.value.code == native.RECON_EINVAL
    plan.close()
