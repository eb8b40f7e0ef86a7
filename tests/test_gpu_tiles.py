"""The z-tile flags of the setup transforms (recon_tile_counts) against counts formed on the host.

The forward z pass transforms and writes only the tiles (one y row, a few consecutive x, every z) whose
deposit bricks hold data, and the overdensity step only the tiles with a cell inside the survey mask;
the parity of the overdensity and of Psi with those tiles skipped is covered by the survey tests.  Here
the counts themselves are checked: the bricks each catalogue touches (the bricks holding a base cell and
their seven upper neighbours, which the CIC footprint reaches) give the grid tiles, and the oracle's
integer mask (reading R9) gives the mask tiles.
"""
import numpy as np
import pytest
import torch

from oracle import recon_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu

BRICK = 16


def touched_bricks(pos, n, box_len, origin):
    i0, _, _ = O.cic_coords(pos, n, box_len, origin)
    nb = n // BRICK
    occ = np.zeros((nb, nb, nb), bool)
    b = i0 // BRICK
    occ[b[:, 2], b[:, 1], b[:, 0]] = True
    t = np.zeros_like(occ)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                t |= np.roll(occ, (dz, dy, dx), axis=(0, 1, 2))
    return t


def live_tiles_from_bricks(t, n, tw):
    col = t.any(axis=0)                                   # [brick y][brick x]
    tiles = np.zeros((n, n // tw), bool)
    for y in range(n):
        for xt in range(n // tw):
            tiles[y, xt] = col[y // BRICK, xt * tw // BRICK:(xt + 1) * tw // BRICK].any()
    return int(tiles.sum())


def mask_tiles(mask, n, tw):
    m = mask.any(axis=0)                                  # [y][x]
    return int(m.reshape(n, n // tw, tw).any(axis=2).sum())


@pytest.mark.parametrize("n,scale", [(64, 0.125), (128, 0.25)])
def test_tile_counts_survey(gpu_lib, n, scale):
    from paper_1504_02591_amd import native
    cat = G.config2(n=n, scale=scale)
    dev = torch.device("cuda", 0)
    plan = native.plan_for(cat)
    plan.paint(native.GAL, torch.from_numpy(cat.gal_pos).to(dev))
    plan.paint(native.RAN, torch.from_numpy(cat.ran_pos).to(dev))
    plan.solve()
    tg, tr, tm, nt = plan.tile_counts()[0]
    plan.close()
    tw = n * n // nt
    assert nt * tw == n * n and tw % BRICK == 0
    eg = live_tiles_from_bricks(touched_bricks(cat.gal_pos, n, cat.box_len, cat.origin), n, tw)
    er = live_tiles_from_bricks(touched_bricks(cat.ran_pos, n, cat.box_len, cat.origin), n, tw)
    grid_r = O.paint(cat.ran_pos, None, n, cat.box_len, cat.origin)
    em = mask_tiles(O.survey_mask(grid_r, cat.mask_tau), n, tw)
    print(f"n={n}: tiles galaxies {tg} (host {eg}), randoms {tr} (host {er}), mask {tm} (host {em}) of {nt}",
          flush=True)
    assert (tg, tr, tm) == (eg, er, em)
    assert 0 < tm < nt


def test_tile_counts_mean_density_box(gpu_lib):
    """Without randoms there is no mask: every tile counts as inside it; a lattice fills every tile."""
    from paper_1504_02591_amd import native
    cat = G.config3(n=64)
    dev = torch.device("cuda", 0)
    plan = native.plan_for(cat)
    plan.paint(native.GAL, torch.from_numpy(cat.gal_pos).to(dev))
    plan.solve()
    tg, tr, tm, nt = plan.tile_counts()[0]
    plan.close()
    assert (tg, tr, tm) == (nt, 0, nt)


def test_batched_surveys_with_different_footprints(gpu_lib):
    """Two survey realisations whose cones point different ways share one plan: each has its own tile
    flags (counts as formed on the host) and its own overdensity, Psi, eps and shifts as the oracle's."""
    from paper_1504_02591_amd import native
    n, s = 64, 64 / 512.0
    cats = [G.survey(n, 3500.0 * s, bias=2.0, growth=0.74, smooth_r=15.0, r_min=1100.0 * s, r_max=1800.0 * s,
                     omega=2.5, n_target=7.0e5 * s ** 3, ran_factor=20, seed_field=301 + 3 * i, seed_gal=302 + 3 * i,
                     seed_ran=303 + 3 * i, axis=ax) for i, ax in enumerate([(1.0, 1.0, 1.0), (-1.0, 0.4, 0.2)])]
    dev = torch.device("cuda", 0)
    gal = np.concatenate([c.gal_pos for c in cats])
    ran = np.concatenate([c.ran_pos for c in cats])
    goff = np.cumsum([0] + [c.gal_pos.shape[0] for c in cats]).astype(np.int64)
    roff = np.cumsum([0] + [c.ran_pos.shape[0] for c in cats]).astype(np.int64)
    c0 = cats[0]
    plan = native.Plan(n, c0.box_len, c0.observer, c0.bias, c0.growth, c0.smooth_r, origin=c0.origin, batch=2,
                       mask_tau=c0.mask_tau, max_objects=ran.shape[0], keep_delta=True)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    plan.paint(native.GAL, to(gal), offsets=to(goff))
    plan.paint(native.RAN, to(ran), offsets=to(roff))
    plan.solve()
    tiles = plan.tile_counts()
    rc, iters, eps = plan.iterate(3, 0.0)
    psi = plan.psi().cpu().numpy()
    delta = plan.delta().cpu().numpy()
    disp = plan.shift(native.GAL, to(gal), offsets=to(goff)).cpu().numpy()
    grid_g, grid_r = plan.grid(native.GAL).cpu().numpy(), plan.grid(native.RAN).cpu().numpy()
    plan.close()
    assert tiles[0][:3] != tiles[1][:3]
    for i, c in enumerate(cats):
        tg, tr, tm, nt = tiles[i]
        tw = n * n // nt
        r = O.reconstruct(c.gal_pos, None, c.ran_pos, None, n, c.box_len, c.origin, c.observer, c.bias, c.growth,
                          c.smooth_r, c.mask_tau, n_passes=3)
        assert np.array_equal(grid_g[i], r["grid_g"]) and np.array_equal(grid_r[i], r["grid_r"])
        assert tg == live_tiles_from_bricks(touched_bricks(c.gal_pos, n, c.box_len, c.origin), n, tw)
        assert tr == live_tiles_from_bricks(touched_bricks(c.ran_pos, n, c.box_len, c.origin), n, tw)
        assert tm == mask_tiles(O.survey_mask(r["grid_r"], c.mask_tau), n, tw)
        e_d = float(np.linalg.norm(delta[i] - r["delta_s"]) / np.linalg.norm(r["delta_s"]))
        e_p = float(np.linalg.norm(psi[i] - r["psi"]) / np.linalg.norm(r["psi"]))
        e_s = float(np.abs(disp[goff[i]:goff[i + 1]] - r["disp_g"]).max())
        print(f"realisation {i}: tiles {tiles[i]}, delta rel L2 {e_d:.2e}, psi rel L2 {e_p:.2e}, "
              f"displacement {e_s:.2e}", flush=True)
        assert e_d < 1e-5 and e_p < 1e-5 and e_s < 1e-4
        np.testing.assert_allclose(eps[i], r["eps"], rtol=1e-4, atol=1e-6)
