"""FP64 CPU oracle for iterative Fourier-space reconstruction with wide-angle RSD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library and
imports nothing from the package; callers hand it NumPy arrays.

Every step is written as the plain definition, in float64 unless the step is
integer-defined, with a library FFT (scipy.fft) as the only primitive.  The
notation follows Burden, Percival & Howlett, "Reconstruction in Fourier space"
(arXiv:1504.02591):

* Lagrangian map x = q + Psi(q)                      -- Sec. 2, eq. (Lagrange)
* overdensity delta = (rho - rho_bar) / rho_bar       -- Sec. 2
* Zel'dovich displacement Psi(k) = i k delta(k)/k^2   -- Sec. 2, eq. (Zeldovich)
* Nusser-Davis equation with the wide-angle RSD term  -- Sec. 2, eq. (Nusser)
* Gaussian smoothing S(k) applied in Fourier space    -- Sec. 3.1
* randoms, separate smoothing, binary survey mask     -- Sec. 3.2
* FFTA starting points                                 -- Sec. 2.2 eq. (approx1), Sec. 4.1 eq. (approx2)
* the iterative RSD removal                           -- Sec. 5.1, eq. (iterative)

Readings taken where the paper is silent or inconsistent (each is restated in
the design notes of the repository):

R1  Transform convention: forward F(k) = sum_x f(x) exp(-i k.x), inverse
    carries 1/N^3.  With it the Zel'dovich solve is Psi(k) = +i k' D(k)/(b k^2),
    which is the sign that makes div Psi = -delta/b (Sec. 6, eq. (delta)).
R2  The RSD correction is added at the galaxy-density level and the sum is
    divided by b: D_{n+1} = D_s + f div[(Psi_n.r)r], Psi_{n+1} = i k' D_{n+1}/(b k^2).
    The fixed point solves div Psi + (f/b) div[(Psi.r)r] = -delta_s/b, i.e.
    eq. (Nusser) with beta = f/b (identical to the printed form when b = 1).
R3  The plane-parallel iterate is D_n = D_s [1 - (-beta mu^2)^(n+1)]/(1 + beta mu^2);
    the sign printed in eq. (itpsi) is reversed with respect to the paper's own
    first two iterates and its Tables 2-3 (n = 0 over-estimates Psi).
R4  Smoothing kernel S(k) = exp(-k^2 R^2 / 2) with the full k^2.
R5  Cloud-in-cell assignment (the paper bins with NGP) in an integer fixed-point
    form so that two independent implementations agree bit for bit.
R6  Grid node (ix,iy,iz) sits at origin + H (ix,iy,iz), H = L/N; arrays are
    indexed [iz][iy][ix] (x fastest); the box is periodic.
R7  Derivative factor k'_j = k_j except k'_j = 0 at the Nyquist index of axis j;
    k^2 and S use the full k; Psi(k = 0) = 0.
R8  alpha = W_g/W_r from the exact integer totals; galaxy and random densities are
    smoothed separately and delta is formed in configuration space.
R9  Binary mask: cell is inside when the exact integer sum of the random grid over
    its 3x3x3 periodic neighbourhood exceeds floor(tau * 27 * W_r / n_occ), where
    n_occ counts cells with a non-zero random deposit.  Cells whose smoothed
    random density is not positive are treated as outside.
R10 Line of sight r = (x - O)/|x - O| per grid node, r = 0 at the observer.
R11 The correction term is not re-smoothed (delta_s is already smoothed).
R12 Convergence: eps_n = ||Psi_n - Psi_{n-1}|| / ||Psi_n|| over all cells and the
    three components; the pass count n counts correction passes (n = 0 is the start).
    Divergence: eps_n non-finite, eps rising on two consecutive passes to a value
    above EPS_FLOOR (rises below it are rounding noise of a converged FP32 iteration),
    or ||Psi_n|| above 100 ||Psi_1|| (the iteration only converges for beta mu^2 < 1,
    eq. (itpsi) and the remark after it).
R13 Shift: galaxies move by -Psi - f (Psi.r) r, randoms by -Psi, with Psi
    interpolated to the object by the same CIC stencil.
R14 FFTA starts with beta in place of f: c = beta/(1+beta) (eq. approx1) or
    3 beta/(7 + 3 beta) (eq. approx2).
R17 Helmholtz split (Sec. 4.1): the projection k_x k_j / k^2 uses the derivative wavenumbers
    (zero at each axis's Nyquist index, R7) and the full k^2; the k = 0 mode (the mean of Psi.x)
    goes to the solenoidal part; the solenoidal part is the remainder (Psi.x) x - irrotational.
R16 NGP option: the paper bins with NGP (Sec. 3.1); node i+1 when the FP32 fraction is >= 1/2.
    The shift keeps the CIC interpolation of R13.
R15 Lognormal option (Sec. 6, eq. logdelta): the smoothed, masked delta_s is replaced by
    ln(max(1 + delta_s, 1e-3)) + C, C = -<ln(max(1 + delta_s, 1e-3))> over all cells (masked
    cells have delta_s = 0 and map to C); the clamp keeps FP32 rounding in empty regions from
    reaching the logarithm's pole.
R18 Relaxed iteration option (not in the paper; it changes the path, not the fixed point):
    D_{n+1} = (1 - w) D_n + w (D_s + f div[(Psi_n.r)r]) with w = 2/(2 + beta).  The pass of
    Sec. 5.1 maps D_n to D_s + T D_n with T D = -beta G^H P G (D/k^2), where G X = (i k'_j X)_j,
    G^H its adjoint and P the pointwise projection v -> (v.r) r.  T is similar to
    -beta (G/|k|)^H P (G/|k|), a symmetric operator with |k'| <= |k| and P a projection, so its
    eigenvalues are real and lie in [-beta, 0]; those of the relaxed pass, 1 - w + w lambda, lie in
    [1 - w(1 + beta), 1 - w], whose largest modulus beta/(2 + beta) is the smallest any w gives.
    The first pass after a non-gradient start (FFTA, learned) has no D_0 to mix with and is the
    plain pass; every other pass, including the first pass of the plain start (D_0 = D_s), is relaxed.
"""
from __future__ import annotations

EPS_FLOOR = 1e-5   # rises of eps below this are not divergence (R12)

import os

import numpy as np
import scipy.fft as sfft

# FFT threads: the host cores this process may use, capped at 16 (one GPU's share of a box)
WORKERS = int(os.environ.get("ORACLE_WORKERS", min(16, len(os.sched_getaffinity(0)))))

FRAC_BITS = 16          # per-axis CIC fraction quantum is 2^-16
WEIGHT_BITS = 32        # weights are stored as integers in units of 2^-32
MAX_WEIGHT = 64.0       # weights must satisfy 0 <= w < 64
MAX_CELL_COORD = 2 ** 30

START_PLAIN, START_FFTA1, START_FFTA2, START_LEARNED = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# Grid frame and wavenumbers (R6, R7)
# ---------------------------------------------------------------------------
def node_positions(n, box_len, origin):
    """Coordinates of every grid node, shape (3, n, n, n) ordered (x, y, z) on [iz][iy][ix]."""
    h = float(box_len) / n
    i = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    return np.stack([origin[0] + h * x, origin[1] + h * y, origin[2] + h * z])


def line_of_sight(n, box_len, origin, observer):
    """Unit vector from the observer to every node (Sec. 2, eq. (Nusser) r-hat), zero at the observer."""
    pos = node_positions(n, box_len, origin)
    rel = pos - np.asarray(observer, dtype=np.float64).reshape(3, 1, 1, 1)
    dist = np.sqrt(np.sum(rel * rel, axis=0))
    out = np.zeros_like(rel)
    nz = dist > 0
    out[:, nz] = rel[:, nz] / dist[nz]
    return out


def wavenumbers(n, box_len):
    """Full wavenumbers (for k^2 and S) and derivative wavenumbers on the rfftn half-spectrum.

    Returns kx, ky, kz, dkx, dky, dkz broadcastable to shape (n, n, n//2+1) of
    an rfftn over axes (z, y, x).
    """
    m_full = np.fft.fftfreq(n, d=1.0 / n)                 # 0..n/2-1, -n/2..-1
    m_half = np.arange(n // 2 + 1, dtype=np.float64)      # 0..n/2
    scale = 2.0 * np.pi / box_len
    k_full = m_full * scale
    k_half = m_half * scale
    d_full = np.where(np.abs(m_full) == n // 2, 0.0, k_full)
    d_half = np.where(m_half == n // 2, 0.0, k_half)
    kz = k_full.reshape(n, 1, 1)
    ky = k_full.reshape(1, n, 1)
    kx = k_half.reshape(1, 1, n // 2 + 1)
    dkz = d_full.reshape(n, 1, 1)
    dky = d_full.reshape(1, n, 1)
    dkx = d_half.reshape(1, 1, n // 2 + 1)
    return kx, ky, kz, dkx, dky, dkz


def fwd(f):
    """Forward real-to-complex transform, exp(-i k.x) convention (R1)."""
    return sfft.rfftn(np.asarray(f, dtype=np.float64), axes=(0, 1, 2), workers=WORKERS)


def inv(fk, n):
    """Inverse complex-to-real transform with the 1/N^3 factor (R1)."""
    return sfft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2), workers=WORKERS)


# ---------------------------------------------------------------------------
# Integer fixed-point cloud-in-cell deposit (Sec. 3.1 binning, R5)
# ---------------------------------------------------------------------------
def cic_coords(pos, n, box_len, origin):
    """Per-axis cell index, 16-bit fraction and exact FP32 fraction of every object.

    u = fl32(fl32(x - o) * s) with s = fl32(n / L); i = floor(u) mod n;
    t = u - floor(u) (exact); tau = floor(t * 2^16).
    Returns (i0 int64 [m,3], tau int64 [m,3], t float32 [m,3]) in (x, y, z) order.
    """
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    s = np.float32(np.float64(n) / np.float64(box_len))
    o = np.asarray(origin, dtype=np.float64).astype(np.float32)
    d = (pos - o).astype(np.float32)
    u = (d * s).astype(np.float32)
    if not np.all(np.isfinite(u)) or np.any(np.abs(u) >= MAX_CELL_COORD):
        raise ValueError("positions must be finite and within 2^30 cells of the box")
    fl = np.floor(u)
    t = (u - fl).astype(np.float32)
    tau = np.floor(t.astype(np.float64) * (1 << FRAC_BITS)).astype(np.int64)
    i0 = np.mod(fl.astype(np.int64), n)
    return i0, tau, t


def quantise_weights(w, m):
    """W_Q = round-half-even(w * 2^32) as int64; w = None means unit weights."""
    if w is None:
        return np.full(m, 1 << WEIGHT_BITS, dtype=np.int64)
    w = np.asarray(w, dtype=np.float32).reshape(-1)
    if w.shape[0] != m:
        raise ValueError("weight count does not match position count")
    if not np.all(np.isfinite(w)) or np.any(w < 0) or np.any(w >= MAX_WEIGHT):
        raise ValueError("weights must be finite and in [0, 64)")
    return np.rint(w.astype(np.float64) * float(1 << WEIGHT_BITS)).astype(np.int64)


def corner_shares(wq, tau):
    """Integer share of every object's weight at its 8 corners.

    Corner (dx,dy,dz) has fraction c = a_x a_y a_z in units of 2^-48 with
    a^0 = 2^16 - tau, a^1 = tau.  Seven corners receive floor(W_Q c / 2^48);
    corner (1,1,1) receives the remainder so each object deposits exactly W_Q.
    Returns a dict {(dx,dy,dz): int64 array}.
    """
    one = np.int64(1 << FRAC_BITS)
    a = {0: one - tau, 1: tau}
    shares = {}
    acc = np.zeros_like(wq)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                if (dx, dy, dz) == (1, 1, 1):
                    continue
                c = a[dx][:, 0] * a[dy][:, 1] * a[dz][:, 2]          # <= 2^48
                c_hi = c >> 24
                c_lo = c & np.int64((1 << 24) - 1)
                part = (wq * c_hi + ((wq * c_lo) >> 24)) >> 24      # floor(W_Q c / 2^48)
                shares[(dx, dy, dz)] = part
                acc = acc + part
    shares[(1, 1, 1)] = wq - acc
    return shares


def _bincount_int64(idx, vals, size):
    """Exact int64 scatter-add: split values into 26-bit halves whose float64 sums stay exact."""
    lo = vals & np.int64((1 << 26) - 1)
    hi = vals >> 26
    s_lo = np.bincount(idx, weights=lo.astype(np.float64), minlength=size)
    s_hi = np.bincount(idx, weights=hi.astype(np.float64), minlength=size)
    if s_lo.max(initial=0) >= 2.0 ** 53 or s_hi.max(initial=0) >= 2.0 ** 53:
        raise OverflowError("per-cell sum too large for the exact split")
    return (s_hi.astype(np.int64) << 26) + s_lo.astype(np.int64)


def paint(pos, w, n, box_len, origin, log=None):
    """Deterministic fixed-point CIC deposit onto an int64 grid [iz][iy][ix] (units of 2^-32).
    log: optional callable taking a progress line per corner."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    m = pos.shape[0]
    grid = np.zeros(n * n * n, dtype=np.int64)
    if m == 0:
        return grid.reshape(n, n, n)
    i0, tau, _ = cic_coords(pos, n, box_len, origin)
    wq = quantise_weights(w, m)
    shares = corner_shares(wq, tau)
    for (dx, dy, dz), part in shares.items():
        ix = (i0[:, 0] + dx) % n
        iy = (i0[:, 1] + dy) % n
        iz = (i0[:, 2] + dz) % n
        flat = (iz * n + iy) * n + ix
        grid += _bincount_int64(flat, part, n * n * n)
        if log:
            log(f"oracle deposit of {m} objects: corner ({dx}, {dy}, {dz}) done")
    return grid.reshape(n, n, n)


def paint_ngp(pos, w, n, box_len, origin):
    """Nearest-grid-point deposit (the paper's binning, Sec. 3.1) in the same fixed point (units 2^-32).

    Node i + 1 (mod n) when the FP32 fraction t = u - floor(u) is at least 1/2, else node i (R16).
    """
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    m = pos.shape[0]
    grid = np.zeros(n * n * n, dtype=np.int64)
    if m == 0:
        return grid.reshape(n, n, n)
    i0, _, t = cic_coords(pos, n, box_len, origin)
    wq = quantise_weights(w, m)
    ii = np.mod(i0 + (t >= np.float32(0.5)).astype(np.int64), n)
    flat = (ii[:, 2] * n + ii[:, 1]) * n + ii[:, 0]
    grid += _bincount_int64(flat, wq, n * n * n)
    return grid.reshape(n, n, n)


# ---------------------------------------------------------------------------
# Totals, smoothing, mask and overdensity (Sec. 2, Sec. 3.1-3.2, R4, R8, R9)
# ---------------------------------------------------------------------------
def totals(grid_g, grid_r=None):
    """Exact integer totals; alpha = W_g / W_r; n_occ = cells with a random deposit."""
    w_g = int(np.sum(grid_g, dtype=np.int64))
    if grid_r is None:
        return {"W_g": w_g, "W_r": 0, "n_occ": 0, "alpha": None}
    w_r = int(np.sum(grid_r, dtype=np.int64))
    n_occ = int(np.count_nonzero(grid_r))
    alpha = float(w_g) / float(w_r) if w_r > 0 else None
    return {"W_g": w_g, "W_r": w_r, "n_occ": n_occ, "alpha": alpha}


def smooth(rho, box_len, smooth_r):
    """Gaussian smoothing in Fourier space: IFFT[S(k) FFT rho], S = exp(-k^2 R^2/2)."""
    n = rho.shape[0]
    kx, ky, kz, _, _, _ = wavenumbers(n, box_len)
    k2 = kx * kx + ky * ky + kz * kz
    s = np.exp(-0.5 * k2 * smooth_r * smooth_r)
    return inv(fwd(rho) * s, n)


def mask_threshold(w_r, n_occ, tau):
    """Integer threshold on the 27-cell random sum (R9)."""
    thr = float(tau) * 27.0 * float(w_r) / float(n_occ)
    return int(np.floor(thr))


def survey_mask(grid_r, tau):
    """Binary survey mask from the exact 3x3x3 periodic box sum of the random grid (R9)."""
    t = totals(grid_r, grid_r)
    if t["n_occ"] == 0:
        raise ValueError("random grid is empty")
    box = np.zeros_like(grid_r)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                box += np.roll(grid_r, shift=(dz, dy, dx), axis=(0, 1, 2))
    return box > mask_threshold(t["W_r"], t["n_occ"], tau)


def overdensity(grid_g, grid_r, box_len, smooth_r, mask_tau=0.1):
    """Smoothed, masked overdensity delta_s (Sec. 2 definition, Sec. 3.2 procedure).

    With randoms: delta_s = m (G - alpha R)/(alpha R) with G, R the separately
    smoothed galaxy and random densities.  Without randoms (periodic box with a
    uniform mean): delta_s = G / rho_bar - 1.
    """
    n = grid_g.shape[0]
    unit = 2.0 ** -WEIGHT_BITS
    g = smooth(grid_g.astype(np.float64) * unit, box_len, smooth_r)
    if grid_r is None:
        w_g = int(np.sum(grid_g, dtype=np.int64))
        if w_g <= 0:
            raise ValueError("total galaxy weight is zero")     # rho_bar = 0: delta undefined
        rho_bar = float(w_g) * unit / float(n ** 3)
        return g / rho_bar - 1.0
    t = totals(grid_g, grid_r)
    if t["alpha"] is None:
        raise ValueError("total random weight is zero")
    if t["W_g"] <= 0:
        raise ValueError("total galaxy weight is zero")         # alpha = 0: delta undefined
    r = smooth(grid_r.astype(np.float64) * unit, box_len, smooth_r)
    m = survey_mask(grid_r, mask_tau) & (r > 0)
    ar = t["alpha"] * r
    out = np.zeros_like(g)
    out[m] = (g[m] - ar[m]) / ar[m]
    return out


# ---------------------------------------------------------------------------
# Zel'dovich solve and the iteration (Sec. 2 eq. (Zeldovich), Sec. 5.1 eq. (iterative))
# ---------------------------------------------------------------------------
LOG_FLOOR = 1e-3   # lower clamp of 1 + delta_s before the logarithm (R15)


def lognormal(delta_s, floor=LOG_FLOOR):
    """Sec. 6, eq. (logdelta): ln(1 + S*delta) + C with C = -<ln(1 + S*delta)> over all cells.

    delta_s is already smoothed (the paper takes the logarithm of the smoothed field so that it never
    reaches -1).  1 + delta_s is clamped below at `floor` (R15).
    """
    t = np.log(np.maximum(1.0 + np.asarray(delta_s, dtype=np.float64), floor))
    return t - t.mean()


def psi_from_density(dk, n, box_len, bias):
    """Psi_j = IFFT[i k'_j D / (b k^2)], Psi(k=0) = 0 (R1, R7).  Returns (3, n, n, n)."""
    kx, ky, kz, dkx, dky, dkz = wavenumbers(n, box_len)
    k2 = kx * kx + ky * ky + kz * kz
    with np.errstate(divide="ignore", invalid="ignore"):
        pot = np.where(k2 > 0, dk / (bias * k2), 0.0)
    return np.stack([inv(1j * d * pot, n) for d in (dkx, dky, dkz)])


def rsd_divergence(u, rhat, box_len):
    """FFT of div[u r-hat] = sum_j i k'_j FFT[u r_j] (the RSD term of eq. (Nusser))."""
    n = u.shape[0]
    _, _, _, dkx, dky, dkz = wavenumbers(n, box_len)
    return sum(1j * d * fwd(u * rhat[j]) for j, d in enumerate((dkx, dky, dkz)))


def ffta_coefficient(start, growth, bias):
    """c of Psi_0 = Psi_p - c (Psi_p.r) r: eq. (approx1) or eq. (approx2) with beta = f/b (R14)."""
    beta = growth / bias
    if start == START_FFTA1:
        return beta / (1.0 + beta)
    if start == START_FFTA2:
        return 3.0 * beta / (7.0 + 3.0 * beta)
    return 0.0


def relax_weight(growth, bias):
    """w = 2/(2 + beta) of the relaxed pass (R18): centres the pass's eigenvalue interval on 0."""
    return 2.0 / (2.0 + growth / bias)


def reconstruct_field(delta_s, box_len, origin, observer, bias, growth,
                      n_passes=None, tol=None, max_iter=50, start=START_PLAIN,
                      start_correction=None, rhat=None, keep=(), log=None, relax=None):
    """Iterative RSD removal from the smoothed redshift-space overdensity.

    delta_s: (n,n,n) float64.  Runs exactly n_passes passes when given, otherwise
    stops at the first n >= 1 with eps_n <= tol (or max_iter).  start selects the
    starting displacement: plain (Psi from delta_s), FFTA-1/FFTA-2, or learned,
    where start_correction is the scalar field Delta added along r-hat.  relax: the
    weight w of the relaxed iteration (R18), None for the paper's pass.
    Returns dict(psi=(3,n,n,n), eps=[eps_1..], passes=n, diverged=bool, D=final density spectrum,
    psi_at={k: Psi_k for the pass counts k listed in keep}).
    """
    n = delta_s.shape[0]
    if rhat is None:
        rhat = line_of_sight(n, box_len, origin, observer)
        if log:
            log("oracle line of sight done")
    d_s = fwd(delta_s)
    psi_p = psi_from_density(d_s, n, box_len, bias)
    u_p = np.sum(psi_p * rhat, axis=0)
    if start == START_PLAIN:
        psi = psi_p
    elif start in (START_FFTA1, START_FFTA2):
        c = ffta_coefficient(start, growth, bias)
        psi = psi_p - c * u_p * rhat
    elif start == START_LEARNED:
        if start_correction is None:
            raise ValueError("learned start needs the correction field")
        psi = psi_p + np.asarray(start_correction, dtype=np.float64) * rhat
    else:
        raise ValueError("unknown start")
    if log:
        log("oracle start done")

    eps_hist = []
    psi_at = {0: psi.copy()} if 0 in keep else {}
    passes = 0
    diverged = False
    norm1 = None
    dk = d_s
    limit = n_passes if n_passes is not None else max_iter
    while passes < limit:
        u = np.sum(psi * rhat, axis=0)
        full = d_s + growth * rsd_divergence(u, rhat, box_len)
        if relax is None or (passes == 0 and start != START_PLAIN):
            dk = full
        else:
            dk = (1.0 - relax) * dk + relax * full   # dk is D_n here (D_s before the first pass)
        psi_new = psi_from_density(dk, n, box_len, bias)
        num = np.sqrt(np.sum((psi_new - psi) ** 2))
        den = np.sqrt(np.sum(psi_new ** 2))
        eps = num / den if den > 0 else 0.0
        psi = psi_new
        passes += 1
        eps_hist.append(float(eps))
        if passes in keep:
            psi_at[passes] = psi.copy()
        if log:
            log(f"oracle pass {passes}: eps {eps:.3e}")
        norm1 = den if norm1 is None else norm1
        if not np.isfinite(eps):
            diverged = True
            break
        if len(eps_hist) >= 3 and eps_hist[-1] > eps_hist[-2] > eps_hist[-3] and eps_hist[-1] > EPS_FLOOR:
            diverged = True
            break
        if passes >= 2 and den > 100.0 * norm1:
            diverged = True
            break
        if n_passes is None and tol is not None and eps <= tol:
            break
    return {"psi": psi, "eps": eps_hist, "passes": passes, "diverged": diverged, "D": dk, "psi_at": psi_at}


# ---------------------------------------------------------------------------
# Shift (Sec. 1: galaxies and randoms moved back along the displacement; R13)
# ---------------------------------------------------------------------------
def gather(field3, pos, box_len, origin):
    """CIC interpolation of a (3,n,n,n) field at positions with the deposit's cell index and FP32 fraction."""
    n = field3.shape[1]
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    i0, _, t = cic_coords(pos, n, box_len, origin)
    t = t.astype(np.float64)
    out = np.zeros((pos.shape[0], 3), dtype=np.float64)
    for dz in (0, 1):
        wz = t[:, 2] if dz else 1.0 - t[:, 2]
        iz = (i0[:, 2] + dz) % n
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1.0 - t[:, 1]
            iy = (i0[:, 1] + dy) % n
            for dx in (0, 1):
                wx = t[:, 0] if dx else 1.0 - t[:, 0]
                ix = (i0[:, 0] + dx) % n
                wgt = wx * wy * wz
                for j in range(3):
                    out[:, j] += wgt * field3[j][iz, iy, ix]
    return out


def shift(psi, pos, box_len, origin, observer, growth, galaxies):
    """Displacement applied to each object: -Psi - f (Psi.r) r for galaxies, -Psi for randoms."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    p = gather(psi, pos, box_len, origin)
    disp = -p
    if galaxies and growth != 0.0:
        rel = pos.astype(np.float64) - np.asarray(observer, dtype=np.float64)
        dist = np.sqrt(np.sum(rel * rel, axis=1))
        rhat = np.zeros_like(rel)
        nz = dist > 0
        rhat[nz] = rel[nz] / dist[nz, None]
        u = np.sum(p * rhat, axis=1)
        disp = disp - growth * u[:, None] * rhat
    return disp


# ---------------------------------------------------------------------------
# Whole pipeline
# ---------------------------------------------------------------------------
def reconstruct(gal_pos, gal_w, ran_pos, ran_w, n, box_len, origin, observer,
                bias, growth, smooth_r, mask_tau=0.1, n_passes=None, tol=None,
                max_iter=50, start=START_PLAIN, start_correction=None, log_transform=False, log=None,
                relax=None):
    """Paint -> overdensity (-> lognormal transform) -> iteration -> shift, all in FP64 (integer deposit).
    log: optional callable taking one progress line per stage and pass."""
    grid_g = paint(gal_pos, gal_w, n, box_len, origin, log=log)
    grid_r = None if ran_pos is None else paint(ran_pos, ran_w, n, box_len, origin, log=log)
    delta_s = overdensity(grid_g, grid_r, box_len, smooth_r, mask_tau)
    if log_transform:
        delta_s = lognormal(delta_s)
    if log:
        log("oracle overdensity done")
    res = reconstruct_field(delta_s, box_len, origin, observer, bias, growth,
                            n_passes=n_passes, tol=tol, max_iter=max_iter,
                            start=start, start_correction=start_correction, log=log, relax=relax)
    res["grid_g"] = grid_g
    res["grid_r"] = grid_r
    res["delta_s"] = delta_s
    res["disp_g"] = shift(res["psi"], gal_pos, box_len, origin, observer, growth, True)
    if ran_pos is not None:
        res["disp_r"] = shift(res["psi"], ran_pos, box_len, origin, observer, growth, False)
    return res


# ---------------------------------------------------------------------------
# Diagnostics (Sec. 4, Table 1; Sec. 5.2, eq. ratio)
# ---------------------------------------------------------------------------
def radial_ratio_stats(psi_ref, psi, rhat, lo=-1.0, hi=3.0):
    """Mean and standard deviation over grid points of (psi_ref . r) / (psi . r), with ratios
    above hi or below lo cut as outliers (Sec. 4, Table 1); cells with psi . r = 0 count as outliers.
    Returns (mean, std, outlier fraction, kept count)."""
    a = np.sum(np.asarray(psi_ref, dtype=np.float64) * rhat, axis=0).ravel()
    b = np.sum(np.asarray(psi, dtype=np.float64) * rhat, axis=0).ravel()
    ok = b != 0
    ratio = np.where(ok, a / np.where(ok, b, 1.0), np.inf)
    keep = ok & (ratio >= lo) & (ratio <= hi)
    r = ratio[keep]
    if r.size == 0:
        return 0.0, 0.0, 1.0, 0
    return float(r.mean()), float(r.std()), float(1.0 - keep.mean()), int(r.size)


def helmholtz_x(psi_x, box_len):
    """Sec. 4.1, eq. (irrotational) and eq. (solenoidal): split of the plane-parallel RSD field
    (Psi.x) x into its irrotational part, IFFT[k_x k_j / k^2 FFT(Psi.x)], and the solenoidal
    remainder (R17).  Returns (irrotational (3,n,n,n), solenoidal (3,n,n,n))."""
    n = psi_x.shape[0]
    kx, ky, kz, dkx, dky, dkz = wavenumbers(n, box_len)
    k2 = kx * kx + ky * ky + kz * kz
    px = fwd(psi_x)
    with np.errstate(divide="ignore", invalid="ignore"):
        proj = np.where(k2 > 0, dkx * px / k2, 0.0)
    irr = np.stack([inv(d * proj, n) for d in (dkx, dky, dkz)])
    sol = -irr
    sol[0] += psi_x
    return irr, sol
