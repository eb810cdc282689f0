"""Plain FP64 implementation of the FFT-based Yamamoto multipole estimator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every step below follows the paper (Bianchi et al. 2015) in its own order:

  * Sec. 2, Eq. (1): the FKP field F = w (n - alpha n_s); alpha normalises the
    weighted randoms to the weighted galaxies; I = int w^2 nbar^2 dr.
  * Sec. 2, Eq. (3): shot noise (1 + alpha) int nbar w^2 L_ell, kept for ell = 0
    only (the paper states it is negligible for ell > 0).
  * Sec. 3, Eq. (5): A_n(k) = int (k.r)^n F(r) e^{ik.r} dr (hats on k and r).
  * Sec. 3, Eqs. (6)-(8): P_0, P_2, P_4 from A_0, A_2, A_4.
  * Sec. 3, Eqs. (9)-(13): the Cartesian split of (k.r)^n into 1 + 6 + 15 grids
    B_ij and C_ijl, one FFT each, contracted with products of k components.
  * Sec. 4: cloud-in-cell assignment on a cubic periodic box, corrected for the
    assignment window following Jing (2005).

Readings where the paper is silent or ambiguous (each is listed in the design
notes of the repository):

  R1  F carries no I^{-1/2}; the result is divided by I once.
  R2  Discrete scalars: alpha = sum_g w / sum_r w; I = alpha sum_r w^2 nbar
      (or sum_g w^2 nbar when norm_from = 1); S = sum_g w^2 + alpha^2 sum_r w^2.
  R3  The LOS of each particle is its own r-hat = (x - observer)/|x - observer|,
      applied before mass assignment.
  R4  Grid nodes sit at box_min + j H, H = L/N, periodic. CIC: i = floor(u),
      weights (1-f, f) on (i, i+1). TSC: i = floor(u + 1/2), d = u - i, weights
      (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2) on (i-1, i, i+1).
  R5  Unnormalised forward DFT with e^{-2 pi i n.j/N}; the sign does not matter
      because only Re[A_0 A_ell^*] enters.
  R6  Mode n = 0 is excluded; bins are b dn <= |n| < (b+1) dn decided by exact
      integer tests on |n|^2, so every mode with a component at -N/2 (the
      Nyquist plane) is excluded as long as nbins dn <= N/2.
  R7  Compensation (Jing 2005): 0 none; 1 divide by W^2 and subtract S;
      2 divide by W^2 and subtract the aliased noise S prod_i C_p(n_i) / W^2,
      W = prod_i sinc^p(pi n_i / N), p = 2 (CIC) or 3 (TSC),
      C_2 = 1 - 2/3 s^2, C_3 = 1 - s^2 + 2/15 s^4, s = sin(pi n_i / N).
  R8  Shell averages count every mode of the full N^3 lattice once.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

CIC = 2
TSC = 3


@dataclass
class Config:
    """Estimator configuration (mirrors the fields of the C configuration struct)."""
    N: int
    box_min: tuple
    L: float
    observer: tuple = (0.0, 0.0, 0.0)
    assign: int = CIC          # 2 = CIC, 3 = TSC
    ell_max: int = 4           # 0, 2, 4 or 6
    los: int = 0               # 0 = per-particle LOS, 1 = fixed +z
    compensate: int = 2        # 0, 1, 2 (reading R7)
    dn: int = 1                # bin width in units of the fundamental mode
    nbins: int = 0             # 0 -> N // (2 dn)
    norm_from: int = 0         # 0 = randoms, 1 = galaxies (reading R2)

    def __post_init__(self):
        if self.nbins == 0:
            self.nbins = self.N // (2 * self.dn)


# ----------------------------------------------------------------------------
# Sec. 2: catalogue scalars
# ----------------------------------------------------------------------------

def catalogue_scalars(w_g, w_r, nbar_g=None, nbar_r=None, norm_from=0):
    """alpha, I and the shot-noise amplitude S (Sec. 2, Eq. 1 and Eq. 3; reading R2)."""
    w_g = np.asarray(w_g, dtype=np.float64)
    w_r = np.asarray(w_r, dtype=np.float64)
    alpha = w_g.sum() / w_r.sum()
    if norm_from == 0:
        I = alpha * np.sum(w_r * w_r * np.asarray(nbar_r, dtype=np.float64))
    else:
        I = np.sum(w_g * w_g * np.asarray(nbar_g, dtype=np.float64))
    S = np.sum(w_g * w_g) + alpha * alpha * np.sum(w_r * w_r)
    return float(alpha), float(I), float(S)


# ----------------------------------------------------------------------------
# Sec. 3: the Cartesian monomials of Eqs. (10)-(13)
# ----------------------------------------------------------------------------

def los_monomials(ell_max):
    """Exponents (a, b, c) with a+b+c in {0, 2, .., ell_max} and their weights.

    (k.r)^n = sum_{a+b+c=n} n!/(a! b! c!) k_x^a k_y^b k_z^c r_x^a r_y^b r_z^c, which is
    Eq. (10) for n = 2 (weights 1 and 2) and Eq. (12) for n = 4 (weights 1, 4, 6, 12);
    n = 6 is the next such decomposition (28 grids), which Sec. 3 notes exists for the
    higher multipoles.
    """
    out = []
    for n in range(0, ell_max + 1, 2):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                c = n - a - b
                coef = math.factorial(n) // (math.factorial(a) * math.factorial(b) * math.factorial(c))
                out.append(((a, b, c), coef))
    return out


def unit_los(pos, observer, los):
    """r-hat of each particle (reading R3); los = 1 fixes it to +z."""
    pos = np.asarray(pos, dtype=np.float64)
    if los == 1:
        rh = np.zeros_like(pos)
        rh[:, 2] = 1.0
        return rh
    d = pos - np.asarray(observer, dtype=np.float64)[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    return d / r[:, None]


# ----------------------------------------------------------------------------
# Sec. 4: mass assignment
# ----------------------------------------------------------------------------

def axis_weights(u, assign):
    """Base index, offsets and weights along one axis (reading R4)."""
    u = np.asarray(u, dtype=np.float64)
    if assign == CIC:
        i = np.floor(u)
        f = u - i
        return i.astype(np.int64), (0, 1), (1.0 - f, f)
    if assign == TSC:
        i = np.floor(u + 0.5)
        d = u - i
        return i.astype(np.int64), (-1, 0, 1), (0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2)
    raise ValueError("assign must be 2 (CIC) or 3 (TSC)")


def grid_units(pos, box_min, L, N):
    """u = (x - box_min) / H with H = L / N, per axis."""
    pos = np.asarray(pos, dtype=np.float64)
    return (pos - np.asarray(box_min, dtype=np.float64)[None, :]) * (N / float(L))


def assign_to_grid(pos, values, cfg: Config):
    """Periodic CIC/TSC deposit of per-particle values onto g[ix, iy, iz] (FP64)."""
    N = cfg.N
    u = grid_units(pos, cfg.box_min, cfg.L, N)
    values = np.asarray(values, dtype=np.float64)
    ix, ox, wx = axis_weights(u[:, 0], cfg.assign)
    iy, oy, wy = axis_weights(u[:, 1], cfg.assign)
    iz, oz, wz = axis_weights(u[:, 2], cfg.assign)
    g = np.zeros(N * N * N, dtype=np.float64)
    for a, dx in enumerate(ox):
        cx = (ix + dx) % N
        for b, dy in enumerate(oy):
            cy = (iy + dy) % N
            wxy = wx[a] * wy[b]
            for c, dz in enumerate(oz):
                cz = (iz + dz) % N
                flat = (cx * N + cy) * N + cz
                g += np.bincount(flat, weights=values * wxy * wz[c], minlength=N * N * N)
    return g.reshape(N, N, N)


def signed_weights(w_g, w_r, alpha):
    """w' = w for galaxies and -alpha w for randoms (Eq. 1 with the I^{-1/2} moved out)."""
    return np.concatenate([np.asarray(w_g, np.float64), -alpha * np.asarray(w_r, np.float64)])


def los_grids(pos, wprime, cfg: Config):
    """The 1, 7 or 22 grids F r-hat^m of Eqs. (11) and (13) (a dict keyed by (a, b, c))."""
    rh = unit_los(pos, cfg.observer, cfg.los)
    grids = {}
    for (a, b, c), _ in los_monomials(cfg.ell_max):
        vals = wprime * rh[:, 0] ** a * rh[:, 1] ** b * rh[:, 2] ** c
        grids[(a, b, c)] = assign_to_grid(pos, vals, cfg)
    return grids


# ----------------------------------------------------------------------------
# Fourier side
# ----------------------------------------------------------------------------

def mode_lattice(N):
    """Integer mode components n_i in [-N/2, N/2) along each FFT axis."""
    return np.round(np.fft.fftfreq(N) * N).astype(np.int64)


def isqrt_array(n2):
    """Exact integer square root of a non-negative int64 array."""
    s = np.floor(np.sqrt(n2.astype(np.float64))).astype(np.int64)
    s = np.where(s * s > n2, s - 1, s)
    s = np.where((s + 1) * (s + 1) <= n2, s + 1, s)
    return s


def window_and_alias(N, assign):
    """Per-axis W_i = sinc^p(pi n/N) and C_p(n) of Jing (2005) (reading R7)."""
    n = mode_lattice(N).astype(np.float64)
    x = np.pi * n / N
    sinc = np.ones_like(x)
    nz = n != 0
    sinc[nz] = np.sin(x[nz]) / x[nz]
    s2 = np.sin(x) ** 2
    p = assign
    if p == CIC:
        C = 1.0 - (2.0 / 3.0) * s2
    else:
        C = 1.0 - s2 + (2.0 / 15.0) * s2 * s2
    return sinc ** p, C


def fft3(grid):
    """Unnormalised forward 3D DFT, e^{-2 pi i n.j/N} (reading R5)."""
    return np.fft.fftn(grid)


@dataclass
class Result:
    k_eff: np.ndarray
    nmodes: np.ndarray
    P: dict                      # ell -> array[nbins]
    noise: np.ndarray            # shell mean of the subtracted noise, / I
    alpha: float
    I: float
    S: float
    sums: dict = field(default_factory=dict)   # raw FP64 shell sums


def amplitudes(grids_k, cfg: Config):
    """A_0, A_2, A_4 on the full lattice from the FFTs of the monomial grids.

    A_n = sum_{|m| = n} coef_m khat^m G_m (Eqs. 10 and 12); khat is undefined at
    n = 0, where A_2 and A_4 are set to 0 (that mode is never binned).
    """
    N = cfg.N
    nv = mode_lattice(N).astype(np.float64)
    nx = nv[:, None, None]
    ny = nv[None, :, None]
    nz = nv[None, None, :]
    kk = np.sqrt(nx * nx + ny * ny + nz * nz)
    kk[0, 0, 0] = 1.0
    kh = (nx / kk, ny / kk, nz / kk)
    A = {0: grids_k[(0, 0, 0)]}
    for n in range(2, cfg.ell_max + 1, 2):
        acc = np.zeros((N, N, N), dtype=np.complex128)
        for (a, b, c), coef in los_monomials(n):
            if a + b + c != n:
                continue
            acc += coef * (kh[0] ** a) * (kh[1] ** b) * (kh[2] ** c) * grids_k[(a, b, c)]
        acc[0, 0, 0] = 0.0
        A[n] = acc
    return A


def shell_sums(A, cfg: Config, S):
    """FP64 shell sums of |A0|^2/W^2, Re[A0 A_n^*]/W^2 and the noise (Eqs. 6-8; R6-R8)."""
    N = cfg.N
    nv = mode_lattice(N)
    n2 = nv[:, None, None] ** 2 + nv[None, :, None] ** 2 + nv[None, None, :] ** 2
    b = isqrt_array(n2) // cfg.dn
    valid = (n2 > 0) & (b < cfg.nbins)
    Wi, Ci = window_and_alias(N, cfg.assign)
    if cfg.compensate == 0:
        inv_w2 = np.ones((N, N, N))
        noise = np.full((N, N, N), S)
    else:
        W = Wi[:, None, None] * Wi[None, :, None] * Wi[None, None, :]
        inv_w2 = 1.0 / (W * W)
        if cfg.compensate == 1:
            noise = np.full((N, N, N), S)
        else:
            C = Ci[:, None, None] * Ci[None, :, None] * Ci[None, None, :]
            noise = S * C * inv_w2
    bv = b[valid]
    nb = cfg.nbins
    sums = {
        "count": np.bincount(bv, minlength=nb).astype(np.int64)[:nb],
        "k": np.bincount(bv, weights=np.sqrt(n2[valid].astype(np.float64)), minlength=nb)[:nb],
        "noise": np.bincount(bv, weights=noise[valid], minlength=nb)[:nb],
    }
    A0 = A[0]
    for n in range(0, cfg.ell_max + 1, 2):
        q = np.real(A0 * np.conj(A[n])) * inv_w2
        sums[f"Q{n}"] = np.bincount(bv, weights=q[valid], minlength=nb)[:nb]
    return sums


def legendre_combination(sums, cfg: Config, I):
    """Eqs. (6)-(8): P0 = <Q0 - N>/I, P2 = 5/2 <3Q2 - Q0>/I, P4 = 9/8 <35Q4 - 30Q2 + 3Q0>/I;
    for ell = 6 the same construction, (2 ell + 1) <A_0 A_{L_ell}^*> / I with
    L_6(mu) = (231 mu^6 - 315 mu^4 + 105 mu^2 - 5)/16: P6 = 13/16 <231Q6 - 315Q4 + 105Q2 - 5Q0>/I."""
    cnt = sums["count"].astype(np.float64)
    ok = cnt > 0
    den = np.where(ok, cnt * I, 1.0)
    P = {0: np.where(ok, (sums["Q0"] - sums["noise"]) / den, 0.0)}
    if cfg.ell_max >= 2:
        P[2] = np.where(ok, 2.5 * (3.0 * sums["Q2"] - sums["Q0"]) / den, 0.0)
    if cfg.ell_max >= 4:
        P[4] = np.where(ok, 1.125 * (35.0 * sums["Q4"] - 30.0 * sums["Q2"] + 3.0 * sums["Q0"]) / den, 0.0)
    if cfg.ell_max >= 6:
        P[6] = np.where(ok, (13.0 / 16.0) * (231.0 * sums["Q6"] - 315.0 * sums["Q4"] + 105.0 * sums["Q2"]
                                             - 5.0 * sums["Q0"]) / den, 0.0)
    kf = 2.0 * np.pi / cfg.L
    k_eff = np.where(ok, kf * sums["k"] / np.where(ok, cnt, 1.0), 0.0)
    noise = np.where(ok, sums["noise"] / den, 0.0)
    return k_eff, P, noise


def wedges(P):
    """Sec. 5: the wedges P_perp (mu in [0, 1/2]) and P_par (mu in [1/2, 1]) from the first
    three even multipoles, P0 -+ 3/8 P2 +- 15/128 P4 (3/8 and 15/128 are the top-hat
    means of L_2 and L_4 over the two ranges); multipoles not measured count as zero."""
    p0 = np.asarray(P[0], np.float64)
    p2 = np.asarray(P[2], np.float64) if 2 in P else np.zeros_like(p0)
    p4 = np.asarray(P[4], np.float64) if 4 in P else np.zeros_like(p0)
    return p0 - 0.375 * p2 + (15.0 / 128.0) * p4, p0 + 0.375 * p2 - (15.0 / 128.0) * p4


def pk_multipoles(gal_pos, gal_w, ran_pos, ran_w, cfg: Config, gal_nbar=None, ran_nbar=None):
    """The whole gridded Yamamoto estimator, in the paper's order (Secs. 2-4).

    Positions are (n, 3) arrays, weights and nbar (n,) arrays; FP32 inputs are
    promoted exactly to FP64.
    """
    alpha, I, S = catalogue_scalars(gal_w, ran_w, gal_nbar, ran_nbar, cfg.norm_from)
    pos = np.concatenate([np.asarray(gal_pos, np.float64), np.asarray(ran_pos, np.float64)])
    wprime = signed_weights(gal_w, ran_w, alpha)
    grids = los_grids(pos, wprime, cfg)
    grids_k = {m: fft3(g) for m, g in grids.items()}
    A = amplitudes(grids_k, cfg)
    sums = shell_sums(A, cfg, S)
    k_eff, P, noise = legendre_combination(sums, cfg, I)
    return Result(k_eff=k_eff, nmodes=sums["count"], P=P, noise=noise,
                  alpha=alpha, I=I, S=S, sums=sums)


def pk_multipoles_streamed(gal_pos, gal_w, ran_pos, ran_w, cfg: Config, gal_nbar=None, ran_nbar=None):
    """Same result as pk_multipoles, holding one monomial grid at a time.

    For grids too large to keep all 22 transforms in memory: A_2 and A_4 are
    accumulated term by term as each grid is assigned and transformed.
    """
    alpha, I, S = catalogue_scalars(gal_w, ran_w, gal_nbar, ran_nbar, cfg.norm_from)
    pos = np.concatenate([np.asarray(gal_pos, np.float64), np.asarray(ran_pos, np.float64)])
    wprime = signed_weights(gal_w, ran_w, alpha)
    rh = unit_los(pos, cfg.observer, cfg.los)
    N = cfg.N
    nv = mode_lattice(N).astype(np.float64)
    nx = nv[:, None, None]
    ny = nv[None, :, None]
    nz = nv[None, None, :]
    kk = np.sqrt(nx * nx + ny * ny + nz * nz)
    kk[0, 0, 0] = 1.0
    A = {}
    for (a, b, c), coef in los_monomials(cfg.ell_max):
        n = a + b + c
        vals = wprime * rh[:, 0] ** a * rh[:, 1] ** b * rh[:, 2] ** c
        Gm = fft3(assign_to_grid(pos, vals, cfg))
        if n == 0:
            A[0] = Gm
            continue
        term = coef * ((nx / kk) ** a) * ((ny / kk) ** b) * ((nz / kk) ** c) * Gm
        del Gm
        if n not in A:
            A[n] = term
        else:
            A[n] += term
        del term
    for n in A:
        if n:
            A[n][0, 0, 0] = 0.0
    sums = shell_sums(A, cfg, S)
    k_eff, P, noise = legendre_combination(sums, cfg, I)
    return Result(k_eff=k_eff, nmodes=sums["count"], P=P, noise=noise,
                  alpha=alpha, I=I, S=S, sums=sums)


def x_transformed_row(pos, wprime, cfg: Config, m, iy, iz):
    """One x-row of the FFT along x of grid m at (iy, iz): used to check sampled rows.

    Only particles whose stencil reaches the row contribute; the row is gridded in
    FP64 and transformed with the library DFT along x.
    """
    N = cfg.N
    u = grid_units(pos, cfg.box_min, cfg.L, N)
    ix, ox, wx = axis_weights(u[:, 0], cfg.assign)
    jy, oy, wy = axis_weights(u[:, 1], cfg.assign)
    jz, oz, wz = axis_weights(u[:, 2], cfg.assign)
    rh = unit_los(pos, cfg.observer, cfg.los)
    a, b, c = m
    vals = np.asarray(wprime, np.float64) * rh[:, 0] ** a * rh[:, 1] ** b * rh[:, 2] ** c
    row = np.zeros(N)
    for bb, dy in enumerate(oy):
        hy = ((jy + dy) % N) == iy
        for cc, dz in enumerate(oz):
            hz = ((jz + dz) % N) == iz
            sel = hy & hz
            if not np.any(sel):
                continue
            for aa, dx in enumerate(ox):
                cx = (ix[sel] + dx) % N
                row += np.bincount(cx, weights=vals[sel] * wx[aa][sel] * wy[bb][sel] * wz[cc][sel],
                                   minlength=N)
    return np.fft.fft(row)


# ----------------------------------------------------------------------------
# Lean forms for the largest grids (N = 512, 1024 on a host)
# ----------------------------------------------------------------------------

def deposit(pos, values, cfg: Config):
    """The same periodic CIC/TSC deposit as assign_to_grid, with the cells and weights of
    several stencil offsets gathered first and summed by one bincount over the grid (for
    catalogues far smaller than the grid, where a dense bincount of N^3 bins per stencil
    offset would dominate the cost; the gathered lists are kept to about N^3 entries)."""
    N = cfg.N
    u = grid_units(pos, cfg.box_min, cfg.L, N)
    values = np.asarray(values, dtype=np.float64)
    ix, ox, wx = axis_weights(u[:, 0], cfg.assign)
    iy, oy, wy = axis_weights(u[:, 1], cfg.assign)
    iz, oz, wz = axis_weights(u[:, 2], cfg.assign)
    g = np.zeros(N * N * N, dtype=np.float64)
    cells, weights = [], []

    def flush():
        if cells:
            g[:] += np.bincount(np.concatenate(cells), weights=np.concatenate(weights), minlength=N * N * N)
            cells.clear()
            weights.clear()
    for a, dx in enumerate(ox):
        cx = (ix + dx) % N
        for b, dy in enumerate(oy):
            cy = (iy + dy) % N
            wxy = wx[a] * wy[b]
            for c, dz in enumerate(oz):
                cz = (iz + dz) % N
                cells.append((cx * N + cy) * N + cz)
                weights.append(values * wxy * wz[c])
                if len(cells) * len(values) >= N * N * N:
                    flush()
    flush()
    return g.reshape(N, N, N)


class _HalfLattice:
    """The binned modes of the half lattice nz in [0, N/2), chunk by chunk of kx planes,
    with every per-mode factor the shell sums need: the flat index of the mode inside its
    chunk, its bin, |n|, k-hat, the multiplicity (1 on nz = 0, 2 elsewhere: the modes
    with nz < 0 are the complex conjugates of those with nz > 0), 1/W^2 and the noise
    factor C/W^2 (or 1). Computed once and reused for every grid."""

    def __init__(self, cfg: Config, planes):
        N = cfg.N
        nv = mode_lattice(N)
        nzv = np.arange(N // 2, dtype=np.int64)
        Wi, Ci = window_and_alias(N, cfg.assign)
        self.chunks = []
        for x0 in range(0, N, planes):
            x1 = min(N, x0 + planes)
            nx = nv[x0:x1][:, None, None]
            ny = nv[None, :, None]
            nz = nzv[None, None, :]
            n2 = (nx * nx + ny * ny + nz * nz).reshape(-1)
            b = isqrt_array(n2) // cfg.dn
            idx = np.nonzero((n2 > 0) & (b < cfg.nbins))[0]
            if idx.size == 0:
                continue
            shape = (x1 - x0, N, N // 2)
            jx, jy, jz = np.unravel_index(idx, shape)
            mx, my, mz = nv[x0:x1][jx], nv[jy], nzv[jz]
            kn = np.sqrt(n2[idx].astype(np.float64))
            mult = np.where(mz == 0, 1.0, 2.0)
            if cfg.compensate == 0:
                inv_w2 = np.ones(idx.size)
                cnoise = np.ones(idx.size)
            else:
                W = Wi[x0:x1][jx] * Wi[jy] * Wi[jz]
                inv_w2 = 1.0 / (W * W)
                cnoise = np.ones(idx.size) if cfg.compensate == 1 else Ci[x0:x1][jx] * Ci[jy] * Ci[jz] * inv_w2
            self.chunks.append(dict(x0=x0, x1=x1, idx=idx, bin=b[idx], k=kn, mult=mult, inv_w2=inv_w2,
                                    cnoise=cnoise, kh=(mx / kn, my / kn, mz / kn)))

    @staticmethod
    def take(grid_k, ch):
        """The values of a half-lattice array at the chunk's binned modes."""
        return grid_k[ch["x0"]:ch["x1"]].reshape(-1)[ch["idx"]]


def _half_spectrum(grid, workers):
    """The transform of a real grid on the half lattice nz in [0, N/2): the library's
    real-input FFT (the same unnormalised e^{-2 pi i n.j/N} transform as fft3)."""
    import scipy.fft as sfft
    N = grid.shape[0]
    return sfft.rfftn(grid, workers=workers)[:, :, :N // 2]


def _workers(workers):
    """Threads of the library FFT: at most 16 (a one-GPU share of a host's cores)."""
    return workers or max(1, min(16, os.cpu_count() or 1))


def pk_multipoles_lean(gal_pos, gal_w, ran_pos, ran_w, cfg: Config, gal_nbar=None, ran_nbar=None,
                       workers=None, planes=16, log=None, max_grids=None):
    """Same result as pk_multipoles, in the memory of about two transformed grids.

    Two facts of the same definition make it lean; the steps are otherwise those of
    pk_multipoles (Secs. 2-4) in the same order:

      * the monomial grids are real, so G_m(-n) = conj G_m(n), and every k-hat monomial
        of even degree is even in k-hat: Re[A_0 A_n^*], W^2, the noise and the bin of -n
        equal those of n. The full-lattice shell sums are the sums over the half lattice
        nz >= 0 with weight 1 on the nz = 0 plane and 2 elsewhere (the plane nz = -N/2 is
        never binned when nbins dn <= N/2);
      * Re[A_0 A_n^*] = sum_{|m| = n} c_m khat^m Re[A_0 G_m^*] (Eqs. 10, 12; khat^m is real)
        is linear in the grids, so the shell sums of Q_n are accumulated grid by grid
        and only A_0 (at the binned modes) and the current G_m are held.

    log(message), if given, is called after the set-up and after each grid; max_grids, if
    given, stops after that many grids (an incomplete result, for timing a sample only).
    """
    assert cfg.nbins * cfg.dn <= cfg.N // 2, "bins must stay below the Nyquist frequency"
    workers = _workers(workers)
    alpha, I, S = catalogue_scalars(gal_w, ran_w, gal_nbar, ran_nbar, cfg.norm_from)
    pos = np.concatenate([np.asarray(gal_pos, np.float64), np.asarray(ran_pos, np.float64)])
    wprime = signed_weights(gal_w, ran_w, alpha)
    rh = unit_los(pos, cfg.observer, cfg.los)
    nb = cfg.nbins
    lat = _HalfLattice(cfg, planes)
    sums = {"count": np.zeros(nb, np.int64), "k": np.zeros(nb), "noise": np.zeros(nb)}
    for n in range(0, cfg.ell_max + 1, 2):
        sums[f"Q{n}"] = np.zeros(nb)
    a0 = []
    if log:
        log("set-up done")
    for i, ((a, b, c), coef) in enumerate(los_monomials(cfg.ell_max)):
        if max_grids is not None and i >= max_grids:
            break
        n = a + b + c
        vals = wprime * rh[:, 0] ** a * rh[:, 1] ** b * rh[:, 2] ** c
        Gm = _half_spectrum(deposit(pos, vals, cfg), workers)
        for j, ch in enumerate(lat.chunks):
            bv, mult = ch["bin"], ch["mult"]
            g = lat.take(Gm, ch)
            if n == 0:
                a0.append(g)
                q = mult * np.real(g * np.conj(g)) * ch["inv_w2"]
                sums["Q0"] += np.bincount(bv, weights=q, minlength=nb)[:nb]
                sums["count"] += np.bincount(bv, weights=mult, minlength=nb)[:nb].astype(np.int64)
                sums["k"] += np.bincount(bv, weights=mult * ch["k"], minlength=nb)[:nb]
                sums["noise"] += np.bincount(bv, weights=mult * S * ch["cnoise"], minlength=nb)[:nb]
                continue
            khx, khy, khz = ch["kh"]
            q = mult * coef * khx ** a * khy ** b * khz ** c * np.real(a0[j] * np.conj(g)) * ch["inv_w2"]
            sums[f"Q{n}"] += np.bincount(bv, weights=q, minlength=nb)[:nb]
        del Gm
        if log:
            log("grid %s done" % ((a, b, c),))
    k_eff, P, noise = legendre_combination(sums, cfg, I)
    return Result(k_eff=k_eff, nmodes=sums["count"], P=P, noise=noise, alpha=alpha, I=I, S=S, sums=sums)


def plane_parallel_multipoles(gal_pos, gal_w, ran_pos, ran_w, cfg: Config, gal_nbar=None, ran_nbar=None,
                              workers=None, planes=16):
    """The estimator with the line of sight fixed to +z, in the plane-parallel form that
    needs one transform: P_l = (2l + 1) <|A_0|^2 L_l(k_z / k) / W^2> / I, minus the noise
    for l = 0 (Sec. 2, Eqs. 2-4 with r-hat = z for every particle, shell-averaged as in
    Eqs. 6-8). It is the cross-path the 22-grid decomposition of Sec. 3 must reduce to
    when every F r-hat^m grid is r_z^n times F. Shell sums over the half lattice as in
    pk_multipoles_lean."""
    from . import direct
    assert cfg.nbins * cfg.dn <= cfg.N // 2, "bins must stay below the Nyquist frequency"
    workers = _workers(workers)
    alpha, I, S = catalogue_scalars(gal_w, ran_w, gal_nbar, ran_nbar, cfg.norm_from)
    pos = np.concatenate([np.asarray(gal_pos, np.float64), np.asarray(ran_pos, np.float64)])
    wprime = signed_weights(gal_w, ran_w, alpha)
    A0 = _half_spectrum(deposit(pos, wprime, cfg), workers)
    nb = cfg.nbins
    ells = tuple(range(0, cfg.ell_max + 1, 2))
    cnt, ks, ns = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    qs = {ell: np.zeros(nb) for ell in ells}
    for ch in _HalfLattice(cfg, planes).chunks:
        bv, mult = ch["bin"], ch["mult"]
        mu = ch["kh"][2]
        p = mult * np.abs(_HalfLattice.take(A0, ch)) ** 2 * ch["inv_w2"]
        cnt += np.bincount(bv, weights=mult, minlength=nb)[:nb]
        ks += np.bincount(bv, weights=mult * ch["k"], minlength=nb)[:nb]
        ns += np.bincount(bv, weights=mult * S * ch["cnoise"], minlength=nb)[:nb]
        for ell in ells:
            qs[ell] += np.bincount(bv, weights=(2 * ell + 1) * p * direct.legendre(ell, mu), minlength=nb)[:nb]
    ok = cnt > 0
    den = I * np.where(ok, cnt, 1.0)
    noise = np.where(ok, ns / den, 0.0)
    P = {ell: np.where(ok, qs[ell] / den - (noise if ell == 0 else 0.0), 0.0) for ell in ells}
    k_eff = np.where(ok, (2.0 * np.pi / cfg.L) * ks / np.where(ok, cnt, 1.0), 0.0)
    return Result(k_eff=k_eff, nmodes=cnt.astype(np.int64), P=P, noise=noise, alpha=alpha, I=I, S=S)


def xy_transformed_column(pos, wprime, cfg: Config, m, kx, ky):
    """The transform along x and y of every plane z of grid m at the mode (kx, ky):
    sum over cells (x, y) of g_m(x, y, z) e^{-2 pi i (kx x + ky y) / N} (unnormalised, the
    sign of fft3), for z = 0 .. N-1, accumulated from each particle's deposits (no grid is
    formed). The weight a particle puts on its cells factorises by axis, so the sum over
    its stencil's (x, y) cells is the product of its two one-axis phase sums."""
    N = cfg.N
    u = grid_units(pos, cfg.box_min, cfg.L, N)
    ix, ox, wx = axis_weights(u[:, 0], cfg.assign)
    iy, oy, wy = axis_weights(u[:, 1], cfg.assign)
    iz, oz, wz = axis_weights(u[:, 2], cfg.assign)
    rh = unit_los(pos, cfg.observer, cfg.los)
    a, b, c = m
    vals = np.asarray(wprime, np.float64) * rh[:, 0] ** a * rh[:, 1] ** b * rh[:, 2] ** c
    px = sum(wx[j] * np.exp(-2j * np.pi * kx * ((ix + d) % N) / N) for j, d in enumerate(ox))
    py = sum(wy[j] * np.exp(-2j * np.pi * ky * ((iy + d) % N) / N) for j, d in enumerate(oy))
    col = np.zeros(N, dtype=np.complex128)
    for j, d in enumerate(oz):
        cz = (iz + d) % N
        v = vals * px * py * wz[j]
        col += np.bincount(cz, weights=v.real, minlength=N) + 1j * np.bincount(cz, weights=v.imag, minlength=N)
    return col
