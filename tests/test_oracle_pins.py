"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than its own code: a
brute-force sum, a closed form, an exact integer identity, or a dense direct
solve of the discretised equation.  None of these tests needs a GPU.
"""
import math
import os

import numpy as np
import pytest

from oracle import recon_oracle as O
from synth import generators as G


# ---------------------------------------------------------------------------
# Helpers written independently of the oracle (explicit loops / dense matrices)
# ---------------------------------------------------------------------------
def brute_dft3(f, sign):
    """Direct triple sum  F(kz,ky,kx) = sum f(z,y,x) exp(sign 2 pi i (kz z + ky y + kx x)/n)."""
    n = f.shape[0]
    idx = np.arange(n)
    e = np.exp(sign * 2j * np.pi * np.outer(idx, idx) / n)
    out = np.zeros((n, n, n), dtype=np.complex128)
    for kz in range(n):
        for ky in range(n):
            for kx in range(n):
                out[kz, ky, kx] = np.sum(f * e[kz][:, None, None] * e[ky][None, :, None] * e[kx][None, None, :])
    return out


def los_loops(n, box_len, origin, observer):
    """Line of sight at each node computed with explicit loops (x fastest in memory)."""
    h = box_len / n
    out = np.zeros((3, n, n, n))
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                r = np.array([origin[0] + h * ix - observer[0], origin[1] + h * iy - observer[1],
                              origin[2] + h * iz - observer[2]])
                d = math.sqrt(r @ r)
                if d > 0:
                    out[:, iz, iy, ix] = r / d
    return out


def dense_operators(n, box_len):
    """Real-space matrices of the spectral gradient (Nyquist derivative zeroed) and Laplacian."""
    m = np.array([i if i < n // 2 else i - n for i in range(n)], dtype=np.float64)
    k1 = 2 * np.pi * m / box_len
    d1 = np.where(np.abs(m) == n // 2, 0.0, k1)
    f1 = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    f3 = np.kron(f1, np.kron(f1, f1))            # acts on vec([z][y][x])
    f3i = np.conj(f3) / n ** 3
    kz = np.repeat(k1, n * n)
    ky = np.tile(np.repeat(k1, n), n)
    kx = np.tile(k1, n * n)
    dz = np.repeat(d1, n * n)
    dy = np.tile(np.repeat(d1, n), n)
    dx = np.tile(d1, n * n)
    grad = [np.real(f3i @ np.diag(1j * d) @ f3) for d in (dx, dy, dz)]
    lap = np.real(f3i @ np.diag(-(kx ** 2 + ky ** 2 + kz ** 2)) @ f3)
    return grad, lap


# ---------------------------------------------------------------------------
# T5: transform convention against a brute-force DFT
# ---------------------------------------------------------------------------
def test_forward_transform_matches_bruteforce_dft():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((8, 8, 8))
    full = brute_dft3(f, -1.0)
    half = O.fwd(f)
    assert half.shape == (8, 8, 5)
    np.testing.assert_allclose(half, full[:, :, :5], rtol=0, atol=1e-11)
    # Hermitian symmetry of a real field's spectrum
    np.testing.assert_allclose(full[1, 2, 3], np.conj(full[-1, -2, -3]), atol=1e-11)


def test_inverse_transform_matches_bruteforce_dft():
    rng = np.random.default_rng(6)
    f = rng.standard_normal((8, 8, 8))
    full = brute_dft3(f, -1.0)
    back = brute_dft3(full, +1.0) / 8 ** 3
    np.testing.assert_allclose(O.inv(O.fwd(f), 8), np.real(back), atol=1e-12)
    np.testing.assert_allclose(np.imag(back), 0.0, atol=1e-12)


def test_parseval_half_spectrum_weights():
    """sum |f|^2 = (1/N^3) sum_half w |F|^2 with w = 2 inside the halved axis (used by the GPU norm)."""
    rng = np.random.default_rng(7)
    n = 16
    f = rng.standard_normal((n, n, n))
    fk = O.fwd(f)
    w = np.full(n // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    assert np.isclose(np.sum(f * f), np.sum(w * np.abs(fk) ** 2) / n ** 3, rtol=1e-12)


# ---------------------------------------------------------------------------
# T1: plane wave -> analytic Zel'dovich displacement (eq. (Zeldovich), eq. (delta))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("modes", [(1, 0, 0), (0, 2, 0), (1, -2, 3), (3, 1, -1)])
def test_plane_wave_displacement_closed_form(modes):
    n, box, amp, ph, b = 16, 400.0, 0.3, 0.7, 1.7
    delta, k0 = G.plane_wave(n, box, modes, amp, ph)
    res = O.reconstruct_field(delta, box, (0, 0, 0), (-1e4, 0, 0), b, 0.0, n_passes=0)
    h = box / n
    i = np.arange(n) * h
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    arg = k0[0] * x + k0[1] * y + k0[2] * z + ph
    k2 = float(k0 @ k0)
    for j in range(3):
        expect = -(amp / (b * k2)) * k0[j] * np.sin(arg)
        np.testing.assert_allclose(res["psi"][j], expect, atol=1e-12)
    # divergence of the closed form returns -delta/b
    div = sum(-(amp / (b * k2)) * k0[j] * k0[j] * np.cos(arg) for j in range(3))
    np.testing.assert_allclose(div, -delta / b, atol=1e-12)


def test_smoothing_of_plane_wave():
    n, box, r = 32, 500.0, 15.0
    delta, k0 = G.plane_wave(n, box, (2, 1, -3), 1.0, 0.3)
    sm = O.smooth(delta, box, r)
    np.testing.assert_allclose(sm, delta * math.exp(-0.5 * float(k0 @ k0) * r * r), atol=1e-12)


# ---------------------------------------------------------------------------
# T2 / T3: f = 0 and the distant-observer closed form of every iterate (eq. (itpsi), R3)
# ---------------------------------------------------------------------------
def test_growth_zero_converges_in_one_pass():
    rng = np.random.default_rng(11)
    d = O.smooth(rng.standard_normal((16, 16, 16)), 300.0, 30.0)
    res = O.reconstruct_field(d, 300.0, (0, 0, 0), (150.3, 151.7, 149.2), 1.3, 0.0, tol=1e-6)
    assert res["passes"] == 1 and res["eps"][0] == 0.0


def _far_observer(axis, box):
    obs = np.array([box / 2] * 3)
    obs[axis] -= 1e12 * box
    return tuple(obs)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_distant_observer_iterates_closed_form(axis):
    n, box, b, f = 16, 400.0, 2.0, 0.74
    beta = f / b
    rng = np.random.default_rng(20 + axis)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 20.0)
    dk_s = O.fwd(delta)
    m = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1)
    kvec = [np.broadcast_to((2 * np.pi / box) * a, (n, n, n // 2 + 1))
            for a in (mh.reshape(1, 1, -1), m.reshape(1, -1, 1), m.reshape(-1, 1, 1))]
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    mlist = [mh.reshape(1, 1, -1), m.reshape(1, -1, 1), m.reshape(-1, 1, 1)]
    dk = [np.where(np.abs(np.broadcast_to(mm, k2.shape)) == n // 2, 0.0, kk) for mm, kk in zip(mlist, kvec)]
    with np.errstate(invalid="ignore", divide="ignore"):
        mu2 = np.where(k2 > 0, dk[axis] ** 2 / k2, 0.0)
    for npass in (0, 1, 2, 5):
        res = O.reconstruct_field(delta, box, (0, 0, 0), _far_observer(axis, box), b, f, n_passes=npass)
        dn = dk_s * (1 - (-beta * mu2) ** (npass + 1)) / (1 + beta * mu2)
        with np.errstate(invalid="ignore", divide="ignore"):
            pot = np.where(k2 > 0, dn / (b * k2), 0.0)
        for j in range(3):
            expect = np.fft.irfftn(1j * dk[j] * pot, s=(n, n, n), axes=(0, 1, 2))
            np.testing.assert_allclose(res["psi"][j], expect, atol=1e-8 * np.abs(expect).max() + 1e-14)


def test_distant_observer_limit_is_kaiser_factor():
    n, box, b, f = 16, 400.0, 1.0, 0.5
    rng = np.random.default_rng(31)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 25.0)
    res = O.reconstruct_field(delta, box, (0, 0, 0), _far_observer(2, box), b, f, n_passes=80)
    m = np.fft.fftfreq(n, d=1.0 / n)
    kz = (2 * np.pi / box) * m.reshape(-1, 1, 1)
    ky = (2 * np.pi / box) * m.reshape(1, -1, 1)
    kx = (2 * np.pi / box) * np.arange(n // 2 + 1).reshape(1, 1, -1)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    dkz = np.where(np.abs(m.reshape(-1, 1, 1)) == n // 2, 0.0, kz)
    with np.errstate(invalid="ignore", divide="ignore"):
        kaiser = np.where(k2 > 0, O.fwd(delta) / (b * k2 * (1 + (f / b) * dkz ** 2 / k2)), 0.0)
    expect = np.fft.irfftn(1j * dkz * kaiser, s=(n, n, n), axes=(0, 1, 2))
    np.testing.assert_allclose(res["psi"][2], expect, atol=1e-10 * np.abs(expect).max())


# ---------------------------------------------------------------------------
# Wide angle: dense direct solve of the discretised eq. (Nusser) with beta = f/b
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("observer", [(31.3, 47.9, 52.1), (-40.0, 130.0, 60.0)])
def test_fixed_point_solves_nusser_davis_equation(observer):
    n, box, b, f = 8, 100.0, 1.5, 0.6
    rng = np.random.default_rng(41)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 12.0)
    grad, lap = dense_operators(n, box)
    rh = los_loops(n, box, (0, 0, 0), observer)
    rvec = [rh[j].ravel() for j in range(3)]
    radial = sum(np.diag(rvec[i]) @ grad[i] for i in range(3))         # phi -> u = (grad phi).r
    rsd = sum(grad[j] @ np.diag(rvec[j]) for j in range(3)) @ radial     # div[(grad phi . r) r]
    a = -b * lap - f * rsd
    rhs = delta.ravel() - delta.mean()
    phi, *_ = np.linalg.lstsq(a, rhs, rcond=None)
    res = O.reconstruct_field(delta, box, (0, 0, 0), observer, b, f, n_passes=90)
    assert res["eps"][-1] < 1e-13
    for j in range(3):
        np.testing.assert_allclose(res["psi"][j].ravel(), grad[j] @ phi, atol=1e-10)


@pytest.mark.parametrize("start", [O.START_FFTA1, O.START_FFTA2])
def test_fixed_point_independent_of_start(start):
    n, box, b, f = 16, 300.0, 2.0, 0.74
    rng = np.random.default_rng(51)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 20.0)
    obs = (150.0, 150.0, 150.0)
    ref = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=60)
    alt = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=60, start=start)
    np.testing.assert_allclose(alt["psi"], ref["psi"], atol=1e-11)


# ---------------------------------------------------------------------------
# Relaxed iteration (R18): same fixed point, per-mode closed form, contraction bound
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 2])
def test_relaxed_distant_observer_iterates_closed_form(axis):
    """Distant observer along an axis: each mode's relaxed pass is the scalar map
    D -> (1 - w) D + w (D_s - beta mu'^2 D), so D_n = D_inf + (1 - w (1 + beta mu'^2))^n (D_s - D_inf)
    with D_inf = D_s / (1 + beta mu'^2) (the Kaiser factor of the plain iteration's limit)."""
    n, box, b, f = 16, 400.0, 2.0, 0.74
    beta = f / b
    w = 2.0 / (2.0 + beta)
    assert O.relax_weight(f, b) == w
    rng = np.random.default_rng(60 + axis)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 20.0)
    dk_s = O.fwd(delta)
    m = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1)
    mlist = [mh.reshape(1, 1, -1), m.reshape(1, -1, 1), m.reshape(-1, 1, 1)]
    kvec = [np.broadcast_to((2 * np.pi / box) * a, (n, n, n // 2 + 1)) for a in mlist]
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    dk = [np.where(np.abs(np.broadcast_to(mm, k2.shape)) == n // 2, 0.0, kk) for mm, kk in zip(mlist, kvec)]
    with np.errstate(invalid="ignore", divide="ignore"):
        mu2 = np.where(k2 > 0, dk[axis] ** 2 / k2, 0.0)
    d_inf = dk_s / (1 + beta * mu2)
    for npass in (1, 2, 5):
        res = O.reconstruct_field(delta, box, (0, 0, 0), _far_observer(axis, box), b, f, n_passes=npass, relax=w)
        dn = d_inf + (1 - w * (1 + beta * mu2)) ** npass * (dk_s - d_inf)
        with np.errstate(invalid="ignore", divide="ignore"):
            pot = np.where(k2 > 0, dn / (b * k2), 0.0)
        for j in range(3):
            expect = np.fft.irfftn(1j * dk[j] * pot, s=(n, n, n), axes=(0, 1, 2))
            np.testing.assert_allclose(res["psi"][j], expect, atol=1e-8 * np.abs(expect).max() + 1e-14)


@pytest.mark.parametrize("observer", [(31.3, 47.9, 52.1), (-40.0, 130.0, 60.0)])
def test_relaxed_fixed_point_solves_nusser_davis_equation(observer):
    """The relaxed passes reach the solution of the discretised eq. (Nusser) found by a dense direct
    solve (the same system as the plain iteration's pin), in fewer passes."""
    n, box, b, f = 8, 100.0, 1.5, 0.6
    rng = np.random.default_rng(41)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 12.0)
    grad, lap = dense_operators(n, box)
    rh = los_loops(n, box, (0, 0, 0), observer)
    rvec = [rh[j].ravel() for j in range(3)]
    radial = sum(np.diag(rvec[i]) @ grad[i] for i in range(3))
    rsd = sum(grad[j] @ np.diag(rvec[j]) for j in range(3)) @ radial
    a = -b * lap - f * rsd
    rhs = delta.ravel() - delta.mean()
    phi, *_ = np.linalg.lstsq(a, rhs, rcond=None)
    res = O.reconstruct_field(delta, box, (0, 0, 0), observer, b, f, n_passes=40, relax=O.relax_weight(f, b))
    assert res["eps"][-1] < 1e-13
    for j in range(3):
        np.testing.assert_allclose(res["psi"][j].ravel(), grad[j] @ phi, atol=1e-10)


def test_relaxed_pass_contracts_by_beta_over_two_plus_beta():
    """Wide angle (observer inside the box): with X = D/|k| the pass is symmetric, so the error
    X_n - X_inf shrinks by at least beta/(2 + beta) per relaxed pass, against at most beta per plain
    pass, which the slowest mode nearly reaches."""
    n, box, b, f = 16, 300.0, 1.0, 0.7
    beta = f / b
    rng = np.random.default_rng(71)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 15.0)
    obs = (140.3, 160.7, 150.2)
    m = np.fft.fftfreq(n, d=1.0 / n)
    mh = np.arange(n // 2 + 1)
    k2 = sum(((2 * np.pi / box) * a) ** 2 for a in (mh.reshape(1, 1, -1), m.reshape(1, -1, 1), m.reshape(-1, 1, 1)))
    inv_k = np.where(k2 > 0, 1.0 / np.sqrt(np.where(k2 > 0, k2, 1.0)), 0.0)
    wgt = np.where((mh == 0) | (mh == n // 2), 1.0, 2.0).reshape(1, 1, -1)

    def xnorm(d):
        return math.sqrt(float(np.sum(wgt * np.abs(d * inv_k) ** 2)))

    x_inf = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=120)["D"]
    for relax, bound in ((O.relax_weight(f, b), beta / (2 + beta)), (None, beta)):
        errs = [xnorm(O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=p, relax=relax)["D"] - x_inf)
                for p in range(1, 7)]
        ratios = [e1 / e0 for e0, e1 in zip(errs, errs[1:])]
        assert max(ratios) <= bound * (1 + 1e-9), (relax, ratios)
        if relax is None:
            assert max(ratios) > 0.5 * beta          # the plain pass is not faster than the bound says
        else:
            assert max(ratios) < 0.6 * beta          # the relaxed one is


@pytest.mark.parametrize("start", [O.START_FFTA2, O.START_LEARNED])
def test_relaxed_iteration_after_non_gradient_start(start):
    """After a non-gradient start the first pass is the plain pass (no D_0 to mix with); the relaxed
    passes that follow reach the plain iteration's fixed point."""
    n, box, b, f = 16, 300.0, 2.0, 0.74
    rng = np.random.default_rng(81)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 20.0)
    corr = 0.1 * O.smooth(rng.standard_normal((n, n, n)), box, 30.0) if start == O.START_LEARNED else None
    obs = (150.0, 120.0, 170.0)
    w = O.relax_weight(f, b)
    one_plain = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=1, start=start, start_correction=corr)
    one_relax = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=1, start=start, start_correction=corr,
                                    relax=w)
    np.testing.assert_array_equal(one_relax["psi"], one_plain["psi"])
    two_plain = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=2, start=start, start_correction=corr)
    two_relax = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=2, start=start, start_correction=corr,
                                    relax=w)
    # the second pass mixes: D_2 = (1 - w) D_1 + w (plain pass from D_1)
    np.testing.assert_allclose(two_relax["D"], (1 - w) * one_plain["D"] + w * two_plain["D"], rtol=0,
                               atol=1e-12 * np.abs(two_plain["D"]).max())
    ref = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=60)
    alt = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=30, start=start, start_correction=corr,
                              relax=w)
    np.testing.assert_allclose(alt["psi"], ref["psi"], atol=1e-11)


def test_ffta_start_changes_only_the_radial_component():
    n, box, b, f = 16, 300.0, 2.0, 0.74
    rng = np.random.default_rng(52)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 20.0)
    obs = (10.0, 20.0, -30.0)
    plain = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=0)
    fa = O.reconstruct_field(delta, box, (0, 0, 0), obs, b, f, n_passes=0, start=O.START_FFTA2)
    rh = los_loops(n, box, (0, 0, 0), obs)
    beta = f / b
    c = 3 * beta / (7 + 3 * beta)                      # eq. (approx2) with beta
    up = np.sum(plain["psi"] * rh, axis=0)
    ua = np.sum(fa["psi"] * rh, axis=0)
    np.testing.assert_allclose(ua, (1 - c) * up, atol=1e-12)
    np.testing.assert_allclose(fa["psi"] - ua * rh, plain["psi"] - up * rh, atol=1e-12)


# ---------------------------------------------------------------------------
# Paper behaviour (Sec. 5, Tables 2-3; values in tests/golden/iteration_ratios.txt): the mean ratio of
# the true to the estimated radial displacement oscillates around 1 with shrinking amplitude for the
# plain start (below 1 after 0 passes, above after 1, ...), and the eq. (approx2) start begins closer
# to 1.  The same pattern must come out of the oracle on a Zel'dovich lattice box.
# ---------------------------------------------------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "iteration_ratios.txt")


def golden_ratio_tables():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            table, sample, start, n, mean, sigma, outl = line.split()
            out.setdefault((int(table), sample, start), []).append((int(n), float(mean)))
    return {k: [m for _, m in sorted(v)] for k, v in out.items()}


def ratio_pattern(plain, ffta0):
    """The three properties of Tables 2-3 (plain-start means by pass count, FFTA start's first mean)."""
    alternates = all((plain[n] - 1.0) * (-1) ** n < 0 for n in range(4))
    shrinks = abs(plain[2] - 1.0) < abs(plain[0] - 1.0) and abs(plain[3] - 1.0) < abs(plain[1] - 1.0)
    ffta_closer = abs(ffta0 - 1.0) < abs(plain[0] - 1.0)
    return alternates, shrinks, ffta_closer


def test_golden_iteration_tables_show_the_pattern():
    tabs = golden_ratio_tables()
    assert sorted(tabs) == [(2, "nbody", "fft"), (2, "nbody", "ffta"), (3, "mock", "fft"), (3, "mock", "ffta")]
    assert len(tabs[(2, "nbody", "fft")]) == 6 and len(tabs[(3, "mock", "fft")]) == 7
    for table, sample in ((2, "nbody"), (3, "mock")):
        assert ratio_pattern(tabs[(table, sample, "fft")], tabs[(table, sample, "ffta")][0]) == (True, True, True)


def test_iterate_ratio_oscillates_as_in_tables():
    cat = G.lattice_box(64, 768.0, (0.0, 0.0, 0.0), 0.75, 7, bias=1.0, smooth_r=10.0)
    args = (cat.n, cat.box_len, cat.origin)
    d_red = O.overdensity(O.paint(cat.gal_pos, None, *args), None, cat.box_len, cat.smooth_r)
    d_real = O.overdensity(O.paint(cat.info["real_pos"], None, *args), None, cat.box_len, cat.smooth_r)
    real = O.reconstruct_field(d_real, cat.box_len, cat.origin, cat.observer, 1.0, 0.0, n_passes=0)
    rh = O.line_of_sight(cat.n, cat.box_len, cat.origin, cat.observer)
    u_real = np.sum(real["psi"] * rh, axis=0)

    def mean_ratio(npass, start):
        it = O.reconstruct_field(d_red, cat.box_len, cat.origin, cat.observer, 1.0, cat.growth, n_passes=npass,
                                 start=start)
        u = np.sum(it["psi"] * rh, axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = u_real / u
        ratio = ratio[np.isfinite(ratio) & (ratio <= 3) & (ratio >= -1)]     # the tables' outlier cut
        return float(ratio.mean())

    plain = [mean_ratio(k, O.START_PLAIN) for k in range(4)]
    ffta0 = mean_ratio(0, O.START_FFTA2)
    tabs = golden_ratio_tables()
    expect = ratio_pattern(tabs[(3, "mock", "fft")], tabs[(3, "mock", "ffta")][0])
    assert ratio_pattern(plain, ffta0) == expect, (plain, ffta0)
    assert plain[0] < 0.95            # the redshift-space start over-estimates the radial displacement


# ---------------------------------------------------------------------------
# T4 / T6: integer CIC deposit
# ---------------------------------------------------------------------------
def test_cic_shares_match_exact_rational_floor():
    rng = np.random.default_rng(60)
    pos = rng.random((200, 3)).astype(np.float32) * 77.0 - 3.0
    w = (rng.random(200) * 63.9).astype(np.float32)
    w[:3] = [0.0, np.float32(2.0 ** -40), np.float32(63.999)]
    n, box = 8, 64.0
    i0, tau, t = O.cic_coords(pos, n, box, (0.0, 0.0, 0.0))
    wq = O.quantise_weights(w, 200)
    shares = O.corner_shares(wq, tau)
    for p in range(200):
        # u recomputed with explicit float32 scalars
        u = [np.float32(np.float32(pos[p, a] - np.float32(0.0)) * np.float32(n / box)) for a in range(3)]
        fl = [math.floor(float(v)) for v in u]
        tq = [math.floor((float(u[a]) - fl[a]) * 65536) for a in range(3)]
        assert [fl[a] % n for a in range(3)] == list(i0[p])
        assert tq == list(tau[p])
        wint = round(float(w[p]) * 2 ** 32)
        if abs(float(w[p]) * 2 ** 32 - math.floor(float(w[p]) * 2 ** 32) - 0.5) < 1e-30:
            wint = int(np.rint(float(w[p]) * 2 ** 32))
        assert wint == wq[p]
        total = 0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    a = [(65536 - tq[k]) if d == 0 else tq[k] for k, d in enumerate((dx, dy, dz))]
                    c = a[0] * a[1] * a[2]
                    exact = (wint * c) // (2 ** 48)          # python big integers
                    if (dx, dy, dz) != (1, 1, 1):
                        assert int(shares[(dx, dy, dz)][p]) == exact
                        total += exact
                    else:
                        last = int(shares[(1, 1, 1)][p])
                        assert 0 <= last - exact <= 7
        assert total + int(shares[(1, 1, 1)][p]) == wint


def test_cic_conserves_weight_and_is_order_independent():
    rng = np.random.default_rng(61)
    n, box = 16, 200.0
    pos = (rng.random((5000, 3)) * 260.0 - 30.0).astype(np.float32)      # includes wrap-around
    w = (rng.random(5000) * 5).astype(np.float32)
    g1 = O.paint(pos, w, n, box, (0.0, 0.0, 0.0))
    perm = rng.permutation(5000)
    g2 = O.paint(pos[perm], w[perm], n, box, (0.0, 0.0, 0.0))
    assert np.array_equal(g1, g2)
    wq = O.quantise_weights(w, 5000)
    assert int(g1.sum()) == int(wq.sum())
    assert abs(int(g1.sum()) * 2.0 ** -32 - float(w.astype(np.float64).sum())) <= 5000 * 2.0 ** -33


def test_cic_single_particle_at_node_and_midpoint():
    n, box = 8, 8.0
    g = O.paint(np.array([[3.0, 4.0, 5.0]], np.float32), None, n, box, (0, 0, 0))
    assert g[5, 4, 3] == 2 ** 32 and g.sum() == 2 ** 32
    g = O.paint(np.array([[7.5, 0.5, 0.5]], np.float32), None, n, box, (0, 0, 0))
    for iz in (0, 1):
        for iy in (0, 1):
            for ix in (7, 0):
                assert g[iz, iy, ix] == 2 ** 29


def test_paint_gather_adjoint():
    rng = np.random.default_rng(62)
    n, box = 16, 100.0
    pos = (rng.random((3000, 3)) * box).astype(np.float32)
    w = (rng.random(3000) * 2).astype(np.float32)
    field = rng.standard_normal((3, n, n, n))
    grid = O.paint(pos, w, n, box, (0, 0, 0)).astype(np.float64) * 2.0 ** -32
    lhs = np.sum(grid * field[0])
    rhs = np.sum(w.astype(np.float64) * O.gather(field, pos, box, (0, 0, 0))[:, 0])
    assert abs(lhs - rhs) <= 2.0 ** -14 * np.sum(np.abs(w)) * np.abs(field[0]).max()


def test_gather_of_linear_field_is_exact():
    n, box = 16, 160.0
    i = np.arange(n) * (box / n)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    field = np.stack([0.3 * x - 0.1 * y + 2.0, 0.7 * y + 0.2 * z, -0.5 * z + 0.01 * x])
    rng = np.random.default_rng(63)
    pos = (5.0 + rng.random((500, 3)) * (box - 20.0)).astype(np.float32)
    got = O.gather(field, pos, box, (0, 0, 0))
    # the stencil sees the FP32 cell coordinate u = fl32(x * fl32(n/L)); map it back exactly
    u = (pos * np.float32(n / box)).astype(np.float32).astype(np.float64)
    p = u * (box / n)
    exp = np.stack([0.3 * p[:, 0] - 0.1 * p[:, 1] + 2.0, 0.7 * p[:, 1] + 0.2 * p[:, 2],
                    -0.5 * p[:, 2] + 0.01 * p[:, 0]], axis=1)
    np.testing.assert_allclose(got, exp, atol=1e-9)


def test_shift_removes_rsd_for_galaxies_only():
    n, box, f = 8, 80.0, 0.6
    psi = np.zeros((3, n, n, n))
    psi[0], psi[1], psi[2] = 1.0, -2.0, 0.5
    obs = (-10.0, 40.0, 40.0)
    pos = np.array([[20.0, 30.0, 50.0], [70.0, 10.0, 5.0]], np.float32)
    dg = O.shift(psi, pos, box, (0, 0, 0), obs, f, True)
    dr = O.shift(psi, pos, box, (0, 0, 0), obs, f, False)
    p = np.array([1.0, -2.0, 0.5])
    for k in range(2):
        r = pos[k].astype(np.float64) - np.array(obs)
        r /= np.linalg.norm(r)
        np.testing.assert_allclose(dg[k], -p - f * (p @ r) * r, atol=1e-12)
        np.testing.assert_allclose(dr[k], -p, atol=1e-12)


# ---------------------------------------------------------------------------
# Mask and overdensity (Sec. 3.2, R9)
# ---------------------------------------------------------------------------
def test_survey_mask_bruteforce():
    rng = np.random.default_rng(70)
    n = 8
    grid = rng.integers(0, 4, size=(n, n, n)).astype(np.int64) * (2 ** 32)
    grid[:3] = 0
    m = O.survey_mask(grid, 0.4)
    w_r, n_occ = int(grid.sum()), int(np.count_nonzero(grid))
    thr = math.floor(0.4 * 27.0 * w_r / n_occ)
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                s = 0
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            s += int(grid[(iz + dz) % n, (iy + dy) % n, (ix + dx) % n])
                assert m[iz, iy, ix] == (s > thr)


def test_uniform_lattice_has_zero_overdensity():
    n, box = 16, 160.0
    i = np.arange(n) * (box / n) + 2.5
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float32)
    g = O.paint(pos, None, n, box, (0, 0, 0))
    d = O.overdensity(g, None, box, 10.0)
    np.testing.assert_allclose(d, 0.0, atol=1e-12)
    r = O.paint(pos, np.full(pos.shape[0], 3.0, np.float32), n, box, (0, 0, 0))
    d2 = O.overdensity(g, r, box, 10.0)
    np.testing.assert_allclose(d2, 0.0, atol=1e-12)


def test_translated_box_gives_the_same_reconstruction():
    """Moving the box origin, the observer and every object by one vector changes nothing the method
    computes (the deposit sees x - origin, the line of sight cell - observer).  Positions on a 1/64
    lattice and an offset of whole units keep every translated coordinate exact in float32, so the
    grids must agree bit for bit and Psi and the shifts to rounding."""
    n, box = 16, 160.0
    rng = np.random.default_rng(21)
    gal = (np.floor(rng.random((400, 3)) * box * 64) / 64).astype(np.float32)
    ran = (np.floor(rng.random((4000, 3)) * box * 64) / 64).astype(np.float32)
    obs = np.array([70.0, 95.0, 60.0])
    off = np.array([-1024.0, 512.0, 256.0])
    a = O.reconstruct(gal, None, ran, None, n, box, (0.0, 0.0, 0.0), tuple(obs), 2.0, 0.7, 15.0, 0.1,
                      n_passes=3)
    b = O.reconstruct((gal + off).astype(np.float32), None, (ran + off).astype(np.float32), None, n, box,
                      tuple(off), tuple(obs + off), 2.0, 0.7, 15.0, 0.1, n_passes=3)
    assert np.array_equal((gal + off).astype(np.float32) - off.astype(np.float32), gal)
    assert np.array_equal(a["grid_g"], b["grid_g"]) and np.array_equal(a["grid_r"], b["grid_r"])
    np.testing.assert_allclose(b["psi"], a["psi"], rtol=0, atol=1e-12 * np.abs(a["psi"]).max())
    np.testing.assert_allclose(b["disp_g"], a["disp_g"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(b["eps"], a["eps"], rtol=1e-10)
    assert np.abs(a["psi"]).max() > 0.1


def test_zero_weight_catalogues_are_refused():
    """delta = (G - alpha R)/(alpha R) needs alpha = W_g/W_r > 0, and G/rho_bar - 1 needs rho_bar > 0
    (Sec. 2, Sec. 3.2): a realisation with no galaxy weight, or no random weight, has no overdensity."""
    n, box = 16, 160.0
    rng = np.random.default_rng(3)
    pos = (rng.random((200, 3)) * box).astype(np.float32)
    g = O.paint(pos, None, n, box, (0, 0, 0))
    r = O.paint(pos, None, n, box, (0, 0, 0))
    empty = O.paint(np.zeros((0, 3), np.float32), None, n, box, (0, 0, 0))
    weightless = O.paint(pos, np.zeros(pos.shape[0], np.float32), n, box, (0, 0, 0))
    assert not empty.any() and not weightless.any()
    for gal in (empty, weightless):
        with pytest.raises(ValueError, match="galaxy weight"):
            O.overdensity(gal, r, box, 10.0)
        with pytest.raises(ValueError, match="galaxy weight"):
            O.overdensity(gal, None, box, 10.0)
    with pytest.raises(ValueError, match="random weight"):
        O.overdensity(g, empty, box, 10.0)
    assert np.isfinite(O.overdensity(g, r, box, 10.0)).all()


def _node_lattice(n, box, weight_of_node):
    """One object on every grid node (box a power of two times n, so every node coordinate and the
    grid scale are exact in float32 and each object's whole weight lands on its own node)."""
    h = box / n
    i = np.arange(n)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    pos = np.stack([x.ravel() * h, y.ravel() * h, z.ravel() * h], axis=1).astype(np.float32)
    w = weight_of_node(x.ravel(), y.ravel(), z.ravel()).astype(np.float32)
    return pos, w


def test_overdensity_with_randoms_closed_form():
    """Pins overdensity() in survey mode (Sec. 2 definition of delta, Sec. 3.2 randoms and mask).

    No smoothing, galaxies of weight 1 + a cos(2 pi m y / L) and randoms of weight 3 on the nodes of
    the half box x < L/2 only.  The galaxy weights average to 1 over the covered nodes, so the
    random-to-galaxy normalisation is alpha = 1/3 and delta_s = w_g / (alpha w_r) - 1 = a cos(2 pi m y/L)
    on the covered nodes, 0 outside the mask.  A denominator of R instead of alpha R, or alpha
    inverted, gives a cos / 3 or 9 (1 + a cos) - 1 and fails."""
    n, box, a, m = 16, 128.0, 0.3, 2
    cover = lambda x, y, z: x < n // 2
    pos_g, w_g = _node_lattice(n, box, lambda x, y, z: 1.0 + a * np.cos(2 * np.pi * m * y / n))
    pos_r, w_r = _node_lattice(n, box, lambda x, y, z: np.full(x.shape, 3.0))
    keep = cover(pos_g[:, 0] / (box / n), None, None)
    g = O.paint(pos_g[keep], w_g[keep], n, box, (0, 0, 0))
    r = O.paint(pos_r[keep], w_r[keep], n, box, (0, 0, 0))
    d = O.overdensity(g, r, box, 0.0, 0.1)
    i = np.arange(n)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    expect = np.where(x < n // 2, a * np.cos(2 * np.pi * m * y / n), 0.0)
    np.testing.assert_allclose(d, expect, rtol=0, atol=2e-7)


def test_overdensity_with_randoms_smoothed_plane_wave():
    """Survey-mode overdensity of a smoothed plane wave (Sec. 3.1 smoothing, Sec. 3.2 separate
    smoothing of galaxies and randoms): galaxies of weight 1 + a cos(k0 . x) and uniform randoms of
    weight 3 on every node; smoothing multiplies the wave by exp(-k0^2 R^2 / 2) and leaves the
    randoms uniform, so delta_s = a exp(-k0^2 R^2/2) cos(k0 . x) everywhere."""
    n, box, a, R = 16, 128.0, 0.25, 9.0
    mx, mz = 1, 2
    pos_g, w_g = _node_lattice(n, box, lambda x, y, z: 1.0 + a * np.cos(2 * np.pi * (mx * x + mz * z) / n))
    pos_r, w_r = _node_lattice(n, box, lambda x, y, z: np.full(x.shape, 3.0))
    g = O.paint(pos_g, w_g, n, box, (0, 0, 0))
    r = O.paint(pos_r, w_r, n, box, (0, 0, 0))
    d = O.overdensity(g, r, box, R, 0.1)
    k2 = (2 * np.pi / box) ** 2 * (mx * mx + mz * mz)
    i = np.arange(n)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    expect = a * np.exp(-0.5 * k2 * R * R) * np.cos(2 * np.pi * (mx * x + mz * z) / n)
    np.testing.assert_allclose(d, expect, rtol=0, atol=2e-7)


def test_bad_inputs_rejected():
    with pytest.raises(ValueError):
        O.paint(np.array([[np.nan, 0, 0]], np.float32), None, 8, 8.0, (0, 0, 0))
    with pytest.raises(ValueError):
        O.paint(np.zeros((1, 3), np.float32), np.array([-1.0], np.float32), 8, 8.0, (0, 0, 0))
    with pytest.raises(ValueError):
        O.overdensity(np.ones((8, 8, 8), np.int64), np.zeros((8, 8, 8), np.int64), 8.0, 1.0)


def test_divergence_beyond_beta_one():
    """Plane-parallel iterates grow as (beta mu^2)^n when beta mu^2 > 1 (remark after eq. (itpsi))."""
    n, box = 16, 300.0
    rng = np.random.default_rng(3)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 30.0)
    res = O.reconstruct_field(delta, box, (0, 0, 0), (150.0, 150.0, -3e9), 1.0, 2.5, tol=1e-6, max_iter=30)
    assert res["diverged"]
    ok = O.reconstruct_field(delta, box, (0, 0, 0), (150.0, 150.0, -3e9), 1.0, 0.9, tol=1e-6, max_iter=400)
    assert not ok["diverged"] and ok["eps"][-1] <= 1e-6


def test_rounding_noise_after_convergence_is_not_divergence():
    """A converged iteration run for a fixed number of passes ends at the rounding floor of eps, where
    eps may rise by chance; below 1e-5 that is not divergence (R12)."""
    n, box = 16, 300.0
    rng = np.random.default_rng(4)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 30.0)
    res = O.reconstruct_field(delta, box, (0, 0, 0), (150.0, 150.0, -3e9), 1.0, 0.5, n_passes=60)
    assert not res["diverged"] and res["passes"] == 60
    assert min(res["eps"]) < 1e-12


def test_lognormal_of_exponential_field_is_its_exponent():
    """Sec. 6, eq. (logdelta): if 1 + delta = exp(g) then ln(1 + delta) + C = g - <g>."""
    rng = np.random.default_rng(21)
    g = 0.4 * rng.standard_normal((8, 8, 8))
    out = O.lognormal(np.exp(g) - 1.0)
    np.testing.assert_allclose(out, g - g.mean(), atol=1e-13)
    assert abs(out.mean()) < 1e-14


def test_lognormal_small_field_second_order():
    """ln(1 + d) + C = t - <t> with t = d - d^2/2 + d^3/3 + O(d^4) (Taylor series, C = -<ln(1 + d)>)."""
    rng = np.random.default_rng(22)
    d = 1e-3 * rng.standard_normal((8, 8, 8))
    t = d - d ** 2 / 2 + d ** 3 / 3
    np.testing.assert_allclose(O.lognormal(d), t - t.mean(), atol=2e-10)


def test_lognormal_clamps_empty_cells():
    d = np.full((4, 4, 4), 0.5)
    d[0, 0, 0] = -1.0          # empty cell: 1 + delta = 0
    t = np.full(d.shape, np.log(1.5))
    t[0, 0, 0] = np.log(O.LOG_FLOOR)
    np.testing.assert_allclose(O.lognormal(d), t - t.mean(), atol=1e-14)


def test_ngp_deposit_brute_force():
    """NGP: every object's whole quantised weight on its nearest node (R16), checked object by object."""
    rng = np.random.default_rng(31)
    n, box = 8, 100.0
    pos = (rng.random((300, 3)) * box - 3.0).astype(np.float32)
    pos[:4] = np.array([[6.25, 0.0, 12.5], [93.75, 99.99, 0.0], [-6.25, 50.0, 18.75], [0.0, 6.2499, 6.2501]],
                       dtype=np.float32)
    w = rng.random(300).astype(np.float32) * 3
    grid = O.paint_ngp(pos, w, n, box, (0.0, 0.0, 0.0))
    ref = np.zeros((n, n, n), dtype=np.int64)
    s = np.float32(n / box)
    for p, wi in zip(pos, w):
        u = [np.float32(np.float32(p[a]) * s) for a in range(3)]
        idx = []
        for a in range(3):
            f = math.floor(float(u[a]))
            frac = float(u[a]) - f
            idx.append((f + (1 if frac >= 0.5 else 0)) % n)
        ref[idx[2], idx[1], idx[0]] += round(float(wi) * 2 ** 32)
    np.testing.assert_array_equal(grid, ref)
    assert grid.sum() == sum(round(float(wi) * 2 ** 32) for wi in w)


def test_radial_ratio_stats_hand_values():
    """Sec. 4, Table 1 statistic: ratio of radial projections, outliers beyond [-1, 3] cut."""
    n = 4
    rhat = O.line_of_sight(n, 40.0, (0, 0, 0), (-100.0, 5.0, 7.0))
    rng = np.random.default_rng(32)
    psi = rng.standard_normal((3, n, n, n))
    m, sd, out, cnt = O.radial_ratio_stats(0.5 * psi, psi, rhat)
    assert abs(m - 0.5) < 1e-14 and sd < 1e-14 and out == 0.0 and cnt == n ** 3
    ref = psi.copy()
    u = np.sum(psi * rhat, axis=0)
    flat = ref.reshape(3, -1)
    # two cells with ratio 5 (cut), one with ratio -2 (cut), the rest ratio 1
    for k, fac in ((0, 5.0), (1, 5.0), (2, -2.0)):
        flat[:, k] += (fac - 1.0) * (u.ravel()[k]) * rhat.reshape(3, -1)[:, k]
    m, sd, out, cnt = O.radial_ratio_stats(ref, psi, rhat)
    assert cnt == n ** 3 - 3 and abs(out - 3 / n ** 3) < 1e-15
    assert abs(m - 1.0) < 1e-12 and sd < 1e-12


def test_helmholtz_split_of_plane_wave():
    """Sec. 4.1: for (Psi.x) x = cos(k.x + p) x the irrotational part is (k_x k_j / k^2) cos(k.x + p)."""
    n, box = 16, 200.0
    for modes in [(1, 0, 0), (2, 3, -1), (0, 4, 1)]:
        f, k0 = G.plane_wave(n, box, modes, 1.0, 0.3)
        irr, sol = O.helmholtz_x(f, box)
        kk = float(k0 @ k0)
        for j in range(3):
            np.testing.assert_allclose(irr[j], k0[0] * k0[j] / kk * f, atol=1e-12)
        np.testing.assert_allclose(sol[0], f - irr[0], atol=1e-14)


def test_helmholtz_parts_are_curl_and_divergence_free():
    """curl of the irrotational part and divergence of the solenoidal part vanish (band-limited field)."""
    n, box = 16, 160.0
    rng = np.random.default_rng(33)
    fk = O.fwd(rng.standard_normal((n, n, n)))
    kx, ky, kz, dkx, dky, dkz = O.wavenumbers(n, box)
    m = 2 * np.pi / box
    band = (np.abs(kx) < (n // 2 - 1) * m) & (np.abs(ky) < (n // 2 - 1) * m) & (np.abs(kz) < (n // 2 - 1) * m)
    f = O.inv(fk * band, n)
    irr, sol = O.helmholtz_x(f, box)
    d = (dkx, dky, dkz)
    ik = [O.fwd(irr[j]) for j in range(3)]
    sk = [O.fwd(sol[j]) for j in range(3)]
    scale = np.abs(fk).max()
    for a, b in ((0, 1), (1, 2), (2, 0)):
        assert np.abs(d[a] * ik[b] - d[b] * ik[a]).max() < 1e-11 * scale
    assert np.abs(sum(d[j] * sk[j] for j in range(3))).max() < 1e-11 * scale
    np.testing.assert_allclose(irr[0] + sol[0], f, atol=1e-13)
    np.testing.assert_allclose(irr[1] + sol[1], 0.0, atol=1e-13)
