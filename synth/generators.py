"""Seeded synthetic catalogues standing in for the paper's N-body and mock data.

Input synthesis only.  This module holds none of the reconstruction's
arithmetic and is imported neither by the FP64 oracle nor by the HIP library:
the tests and the benchmark call it and pass the arrays it returns to both.

The paper measures on a GADGET-2 N-body box (Sec. 3.1) and on PTHalo BOSS DR11
CMASS-North mocks (Sec. 3.2); neither is available, so these catalogues stand
in for them with the same kind of structure: a Gaussian linear field with
P(k) = A k / (1 + (k/0.02)^3) normalised to sigma_8 = 0.8, objects displaced
by the linear Lagrangian displacement of that field (Sec. 2, eq. (Lagrange)),
redshift-space positions s = x + f (Psi.r) r along each object's own line of
sight, and uniform randoms inside the survey geometry.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft
from scipy import integrate

SIGMA8 = 0.8
K_TURN = 0.02
WORKERS = min(16, len(os.sched_getaffinity(0)))


@dataclass
class Catalogue:
    """Galaxies, randoms and the geometry they were drawn for."""
    gal_pos: np.ndarray
    ran_pos: np.ndarray | None
    n: int
    box_len: float
    origin: tuple
    observer: tuple
    bias: float
    growth: float
    smooth_r: float
    mask_tau: float = 0.1
    gal_w: np.ndarray | None = None
    ran_w: np.ndarray | None = None
    info: dict = field(default_factory=dict)

    def params(self):
        return dict(n=self.n, box_len=self.box_len, origin=self.origin, observer=self.observer,
                    bias=self.bias, growth=self.growth, smooth_r=self.smooth_r, mask_tau=self.mask_tau)


def _shape_pk(k):
    return k / (1.0 + (k / K_TURN) ** 3)


def power_amplitude(sigma8=SIGMA8, radius=8.0):
    """A such that the top-hat variance at 8 Mpc/h of A k/(1+(k/0.02)^3) equals sigma8^2."""
    def integrand(lnk):
        k = math.exp(lnk)
        x = k * radius
        w = 3.0 * (math.sin(x) - x * math.cos(x)) / x ** 3 if x > 1e-4 else 1.0 - x * x / 10.0
        return k ** 3 * _shape_pk(k) * w * w / (2.0 * math.pi ** 2)
    val, _ = integrate.quad(integrand, math.log(1e-6), math.log(50.0), limit=500)
    return sigma8 ** 2 / val


def linear_field(n, box_len, seed, want_psi=True, dtype=np.float64, log=None):
    """Gaussian linear density field and its linear displacement on an n^3 grid.

    White noise w ~ N(0,1) -> F_k = FFT(w) sqrt(P(k) n^3 / L^3) with F_0 = 0.
    Arrays are indexed [iz][iy][ix].  Returns (delta, psi or None); psi has shape (3,n,n,n).
    """
    rng = np.random.default_rng(seed)
    ctype = np.complex128 if dtype == np.float64 else np.complex64
    wn = rng.standard_normal((n, n, n), dtype=dtype)
    fk = sfft.rfftn(wn, workers=WORKERS).astype(ctype, copy=False)
    del wn
    if log:
        log(f"white noise on {n}^3 drawn and transformed")
    amp = power_amplitude()
    mf = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1, dtype=np.float64)
    sc = 2.0 * math.pi / box_len
    kz = (mf * sc).reshape(n, 1, 1)
    ky = (mf * sc).reshape(1, n, 1)
    kx = (mh * sc).reshape(1, 1, n // 2 + 1)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.sqrt(amp * _shape_pk(kk) * n ** 3 / box_len ** 3)
    scale[0, 0, 0] = 0.0
    fk *= scale.astype(dtype)
    delta = sfft.irfftn(fk, s=(n, n, n), workers=WORKERS).astype(dtype, copy=False)
    if log:
        log("linear density field formed")
    psi = None
    if want_psi:
        k2 = kx * kx + ky * ky + kz * kz
        k2[0, 0, 0] = 1.0
        dz = np.where(np.abs(mf) == n // 2, 0.0, mf * sc).reshape(n, 1, 1)
        dy = np.where(np.abs(mf) == n // 2, 0.0, mf * sc).reshape(1, n, 1)
        dx = np.where(mh == n // 2, 0.0, mh * sc).reshape(1, 1, n // 2 + 1)
        psi = np.empty((3, n, n, n), dtype=dtype)
        for j, d in enumerate((dx, dy, dz)):
            psi[j] = sfft.irfftn(fk * (1j * d / k2).astype(ctype), s=(n, n, n), workers=WORKERS)
            if log:
                log(f"linear displacement component {j} formed")
    return delta, psi


def _trilinear(field3, pos, n, box_len):
    """Periodic trilinear interpolation of a (3,n,n,n) grid field at positions [m,3] (box origin 0)."""
    u = pos.astype(np.float64) * (n / box_len)
    i0 = np.floor(u).astype(np.int64)
    t = u - i0
    out = np.zeros((pos.shape[0], 3))
    for dz in (0, 1):
        wz = t[:, 2] if dz else 1 - t[:, 2]
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1 - t[:, 1]
            for dx in (0, 1):
                wx = t[:, 0] if dx else 1 - t[:, 0]
                ix = (i0[:, 0] + dx) % n
                iy = (i0[:, 1] + dy) % n
                iz = (i0[:, 2] + dz) % n
                for j in range(3):
                    out[:, j] += wx * wy * wz * field3[j][iz, iy, ix]
    return out


def _unit(v):
    d = np.sqrt(np.sum(v * v, axis=1, keepdims=True))
    return np.divide(v, d, out=np.zeros_like(v), where=d > 0)


# ---------------------------------------------------------------------------
# Periodic lattice box (the N-body stand-in)
# ---------------------------------------------------------------------------
def lattice_box(n, box_len, observer, growth, seed_field, seed_randoms=None, ran_factor=0,
                bias=1.0, smooth_r=10.0, n_part=None):
    """Lattice particles moved by their linear displacement, then redshift-shifted.

    x = q + Psi_L(q);  s = x + f (Psi_L(q).r(x)) r(x), wrapped into [0, L).
    Randoms (ran_factor * n_part^3) are uniform in the periodic box.
    """
    n_part = n if n_part is None else n_part
    _, psi = linear_field(n_part, box_len, seed_field)
    h = box_len / n_part
    i = np.arange(n_part, dtype=np.float64) * h
    qz, qy, qx = np.meshgrid(i, i, i, indexing="ij")
    q = np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)
    p = np.stack([psi[0].ravel(), psi[1].ravel(), psi[2].ravel()], axis=1)
    x = q + p
    rh = _unit(x - np.asarray(observer, dtype=np.float64))
    s = x + growth * np.sum(p * rh, axis=1, keepdims=True) * rh
    s = np.mod(s, box_len)
    s = np.where(s >= box_len, s - box_len, s)
    ran = None
    if ran_factor:
        rng = np.random.default_rng(seed_randoms)
        ran = (rng.random((ran_factor * n_part ** 3, 3)) * box_len).astype(np.float32)
        ran = np.where(ran >= np.float32(box_len), np.float32(0.0), ran)
    return Catalogue(gal_pos=s.astype(np.float32), ran_pos=ran, n=n, box_len=box_len,
                     origin=(0.0, 0.0, 0.0), observer=tuple(float(v) for v in observer),
                     bias=bias, growth=growth, smooth_r=smooth_r,
                     info=dict(kind="lattice", n_part=n_part, seed_field=seed_field,
                               seed_randoms=seed_randoms,
                               real_pos=np.mod(x, box_len).astype(np.float32)))


def lattice_box_large(n, box_len, observer, growth, seed_field, bias=1.0, smooth_r=10.0, slab=32,
                      field_dtype=np.float64, log=None):
    """lattice_box without randoms for large n (the 1024^3 lattice): the same draws and arithmetic
    per object, but the positions are formed slab by slab of z planes (slabs in parallel threads) into
    one float32 array, so that only the linear field, its displacement and a few slabs of float64
    temporaries are held at once.  field_dtype=np.float32 draws the linear field in single precision
    (another, equally valid realisation; half the memory and time at 1024^3)."""
    from concurrent.futures import ThreadPoolExecutor
    _, psi = linear_field(n, box_len, seed_field, dtype=field_dtype, log=log)
    if log:
        log(f"linear field and displacement on {n}^3 drawn")
    h = box_len / n
    obs = np.asarray(observer, dtype=np.float64)
    out = np.empty((n ** 3, 3), dtype=np.float32)
    i = np.arange(n, dtype=np.float64) * h

    def one(z0):
        z1 = min(n, z0 + slab)
        qz, qy, qx = np.meshgrid(i[z0:z1], i, i, indexing="ij")
        q = np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)
        p = np.stack([psi[0, z0:z1].ravel(), psi[1, z0:z1].ravel(), psi[2, z0:z1].ravel()], axis=1)
        x = q + p
        rh = _unit(x - obs)
        s = x + growth * np.sum(p * rh, axis=1, keepdims=True) * rh
        s = np.mod(s, box_len)
        s = np.where(s >= box_len, s - box_len, s)
        out[z0 * n * n:z1 * n * n] = s

    with ThreadPoolExecutor(WORKERS) as ex:
        list(ex.map(one, range(0, n, slab)))
    del psi
    return Catalogue(gal_pos=out, ran_pos=None, n=n, box_len=box_len, origin=(0.0, 0.0, 0.0),
                     observer=tuple(float(v) for v in observer), bias=bias, growth=growth, smooth_r=smooth_r,
                     info=dict(kind="lattice", n_part=n, seed_field=seed_field))


def config1():
    """Oracle-sized periodic box: 64^3 grid, L = 1000, f = 0.7, b = 1, observer (-1000, 500, 500), R = 10."""
    return lattice_box(64, 1000.0, (-1000.0, 500.0, 500.0), 0.7, 101, 102, ran_factor=5,
                       bias=1.0, smooth_r=10.0)


def config3(n=128, log=None):
    """Precision-study box: L = 2000, f = 0.76, b = 1, no randoms, observer 5000 Mpc/h from the centre
    (n^3 lattice particles; the slab-wise generator above 256^3)."""
    if n > 256:
        return lattice_box_large(n, 2000.0, (-4000.0, 1000.0, 1000.0), 0.76, 301, bias=1.0, smooth_r=10.0,
                                 slab=max(1, 4096 // n), field_dtype=np.float32, log=log)
    return lattice_box(n, 2000.0, (-4000.0, 1000.0, 1000.0), 0.76, 301, None, ran_factor=0,
                       bias=1.0, smooth_r=10.0)


# ---------------------------------------------------------------------------
# Survey cone (the mock-catalogue stand-in)
# ---------------------------------------------------------------------------
def _rotation_to(axis):
    """Rotation matrix taking +z to the unit vector axis."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(z, a)
    c = float(np.dot(z, a))
    if np.linalg.norm(v) < 1e-12:
        return np.eye(3) if c > 0 else np.diag([1.0, -1.0, -1.0])
    vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    return np.eye(3) + vx + vx @ vx * (1.0 / (1.0 + c))


def in_survey(pos, observer, axis, cos_max, r_min, r_max, box_len):
    rel = pos - np.asarray(observer, dtype=np.float64)
    d = np.sqrt(np.sum(rel * rel, axis=1))
    a = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    with np.errstate(invalid="ignore", divide="ignore"):
        cos = (rel @ a) / d
    inside_box = np.all((pos >= 0.0) & (pos < box_len), axis=1)
    return (d >= r_min) & (d <= r_max) & (cos >= cos_max) & inside_box


def survey(n, box_len, bias, growth, smooth_r, r_min, r_max, omega, n_target, ran_factor,
           seed_field, seed_gal, seed_ran, observer=None, axis=(1.0, 1.0, 1.0)):
    """Poisson-sampled galaxies in a cone shell with redshift-space distortions, plus randoms.

    Per cell: Poisson(lambda max(0, 1 + b delta_L)) objects placed uniformly in
    the cell, lambda set so the expected count inside the shell is n_target.
    s = x + f (Psi_L(x).r) r with Psi_L interpolated trilinearly; galaxies whose s
    leaves the survey are dropped.  Randoms: ran_factor * N_g uniform in the survey.
    """
    observer = (box_len / 2,) * 3 if observer is None else observer
    obs = np.asarray(observer, dtype=np.float64)
    cos_max = 1.0 - omega / (2.0 * math.pi)
    delta, psi = linear_field(n, box_len, seed_field, dtype=np.float32)
    h = box_len / n
    rng = np.random.default_rng(seed_gal)
    # cells whose centre lies in the survey (slab by slab to bound memory)
    i = (np.arange(n, dtype=np.float64) + 0.5) * h
    cy, cx = np.meshgrid(i, i, indexing="ij")
    flat_xy = np.stack([cx.ravel(), cy.ravel()], axis=1)
    sel_cells, sel_weight = [], []
    for iz in range(n):
        d = np.sqrt((flat_xy[:, 0] - obs[0]) ** 2 + (flat_xy[:, 1] - obs[1]) ** 2 + (i[iz] - obs[2]) ** 2)
        if d.min() > r_max + h or d.max() < r_min - h:
            continue
        ctr = np.column_stack([flat_xy, np.full(flat_xy.shape[0], i[iz])])
        ok = in_survey(ctr, obs, axis, cos_max, r_min, r_max, box_len)
        idx = np.nonzero(ok)[0]
        if idx.size == 0:
            continue
        wgt = np.maximum(0.0, 1.0 + bias * delta[iz].ravel()[idx].astype(np.float64))
        sel_cells.append(iz * n * n + idx)
        sel_weight.append(wgt)
    cells = np.concatenate(sel_cells)
    wgt = np.concatenate(sel_weight)
    lam = wgt * (n_target / wgt.sum())
    counts = rng.poisson(lam)
    cell_of = np.repeat(cells, counts)
    ix = cell_of % n
    iy = (cell_of // n) % n
    iz = cell_of // (n * n)
    x = np.stack([ix, iy, iz], axis=1).astype(np.float64) * h + rng.random((cell_of.size, 3)) * h
    p = _trilinear(psi, x, n, box_len)
    rh = _unit(x - obs)
    s = x + growth * np.sum(p * rh, axis=1, keepdims=True) * rh
    keep = in_survey(s, obs, axis, cos_max, r_min, r_max, box_len)
    gal = s[keep].astype(np.float32)
    n_g = gal.shape[0]
    # randoms uniform in the survey volume
    rrng = np.random.default_rng(seed_ran)
    rot = _rotation_to(axis)
    want = ran_factor * n_g
    parts, have = [], 0
    while have < want:
        m = int((want - have) * 1.02) + 1024
        r = (r_min ** 3 + rrng.random(m) * (r_max ** 3 - r_min ** 3)) ** (1.0 / 3.0)
        ct = 1.0 - rrng.random(m) * (1.0 - cos_max)
        st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
        ph = 2.0 * math.pi * rrng.random(m)
        dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1) @ rot.T
        pts = obs + r[:, None] * dirs
        ok = np.all((pts >= 0.0) & (pts < box_len), axis=1)
        pts = pts[ok].astype(np.float32)
        ok = np.all((pts >= np.float32(0.0)) & (pts < np.float32(box_len)), axis=1)
        parts.append(pts[ok][: want - have])
        have += parts[-1].shape[0]
    ran = np.concatenate(parts) if parts else np.zeros((0, 3), np.float32)
    info = dict(kind="survey", n_target=n_target, n_gal=int(n_g), n_ran=int(ran.shape[0]),
                n_sampled=int(cell_of.size), r_min=r_min, r_max=r_max, omega=omega,
                seeds=(seed_field, seed_gal, seed_ran))
    return Catalogue(gal_pos=gal, ran_pos=ran, n=n, box_len=box_len, origin=(0.0, 0.0, 0.0),
                     observer=tuple(float(v) for v in obs), bias=bias, growth=growth,
                     smooth_r=smooth_r, info=info)


def config2(n=512, scale=1.0, seeds=(201, 202, 203), n_target=7.0e5, ran_factor=50):
    """Survey-like 512^3 / 3500 Mpc/h box, observer at the centre, cone of 2.5 sr, 1100-1800 Mpc/h.

    scale < 1 shrinks the box and the shell together (same cell size when n is scaled too).
    """
    return survey(n, 3500.0 * scale, bias=2.0, growth=0.74, smooth_r=15.0,
                  r_min=1100.0 * scale, r_max=1800.0 * scale, omega=2.5,
                  n_target=n_target * scale ** 3, ran_factor=ran_factor,
                  seed_field=seeds[0], seed_gal=seeds[1], seed_ran=seeds[2])


def config4_realisation(i, n=256):
    """One realisation of the batched workload: 256^3, L = 1500, log-uniform galaxy count in [1e5, 1e6]."""
    rng = np.random.default_rng(40000 + 3 * i)
    n_g = float(np.exp(rng.uniform(math.log(1e5), math.log(1e6))))
    s = 1500.0 / 3500.0
    return survey(n, 1500.0, bias=2.0, growth=0.74, smooth_r=15.0, r_min=1100.0 * s,
                  r_max=1800.0 * s, omega=2.5, n_target=n_g, ran_factor=50,
                  seed_field=40000 + 3 * i, seed_gal=40001 + 3 * i, seed_ran=40002 + 3 * i)


def config5_realisation(i, train=True, n=256, ran_factor=50):
    """Training / test realisation for the learned start at the 512^3 cell size (L = 1750 for 256^3)."""
    base = 50000 if train else 60000
    return config2(n=n, scale=n / 512.0, seeds=(base + 3 * i, base + 3 * i + 1, base + 3 * i + 2))


def plane_wave(n, box_len, modes, amp, phase, origin=(0.0, 0.0, 0.0)):
    """delta(x) = amp cos(k0.x + phase) on the grid nodes with k0 = 2 pi modes / L."""
    h = box_len / n
    i = np.arange(n, dtype=np.float64) * h
    z, y, x = np.meshgrid(i + origin[2], i + origin[1], i + origin[0], indexing="ij")
    k0 = 2.0 * math.pi * np.asarray(modes, dtype=np.float64) / box_len
    return amp * np.cos(k0[0] * x + k0[1] * y + k0[2] * z + phase), k0


def random_positions(m, box_len, seed, lo=0.0, hi=None):
    """Uniform FP32 positions in [lo, hi)^3 (hi defaults to box_len)."""
    hi = box_len if hi is None else hi
    rng = np.random.default_rng(seed)
    return (lo + rng.random((m, 3)) * (hi - lo)).astype(np.float32)
