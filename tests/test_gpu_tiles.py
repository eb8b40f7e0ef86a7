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
