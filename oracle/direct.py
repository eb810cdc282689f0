"""Direct-summation cross-paths for the oracle (no grids-plus-FFT, no Cartesian split).

TEST INFRASTRUCTURE ONLY (see the package docstring).

These evaluate the Yamamoto amplitudes of Sec. 2, Eq. (4) mode by mode as plain
sums over particles, with the Legendre polynomial of k-hat . r-hat evaluated
directly, so that they check the FFT decomposition of Sec. 3 (Eqs. 10-13) and
the Legendre combinations of Eqs. (6)-(8) without sharing their arithmetic:

  interpolated-phase sum  A(n) = sum_p w'_p f(mu_p) sum_c K(u_p - c) e^{-2 pi i n.c/N}
                          with the assignment kernel K written as a function of the
                          distance to a node (not as per-cell weight lists). Sec. 3
                          states that the FFT decomposition adds no approximation, so
                          this equals the gridded estimator to rounding.
  sum-gal (Sec. 4)        A(n) = sum_p w'_p f(mu_p) e^{-i k.(x_p - box_min)}; equal to the
                          gridded estimator for CIC when every particle sits on a node.
  sum-grid (Sec. 4)       the DFT of a grid by direct summation over its cells.
"""
from __future__ import annotations

import numpy as np


def kernel(s, assign):
    """Assignment kernel as a function of the distance s (in cells) to a node.

    CIC: max(0, 1 - |s|).  TSC: 3/4 - s^2 for |s| <= 1/2, (3/2 - |s|)^2 / 2 for
    1/2 < |s| < 3/2, 0 beyond.
    """
    a = np.abs(s)
    if assign == 2:
        return np.clip(1.0 - a, 0.0, None)
    inner = 0.75 - a * a
    outer = 0.5 * (1.5 - a) ** 2
    return np.where(a <= 0.5, inner, np.where(a < 1.5, outer, 0.0))


def legendre(ell, mu):
    if ell == 0:
        return np.ones_like(mu)
    if ell == 2:
        return 0.5 * (3.0 * mu * mu - 1.0)
    if ell == 4:
        m2 = mu * mu
        return (35.0 * m2 * m2 - 30.0 * m2 + 3.0) / 8.0
    if ell == 6:
        m2 = mu * mu
        return (((231.0 * m2 - 315.0) * m2 + 105.0) * m2 - 5.0) / 16.0
    raise ValueError(ell)


def _axis_phase(u, N, assign, n=None):
    """phi[p, j] = sum_c K(u_p - c) e^{-2 pi i n_j c / N} for the frequencies n_j in
    0..N-1 (all of them by default; any integer c)."""
    base = np.floor(u).astype(np.int64)
    n = np.arange(N) if n is None else np.asarray(n, np.int64)
    out = np.zeros((u.shape[0], len(n)), dtype=np.complex128)
    for off in range(-2, 3):
        c = base + off
        k = kernel(u - c, assign)
        out += k[:, None] * np.exp(-2j * np.pi * np.outer(c, n) / N)
    return out


def lattice_modes(N, dn, nbins):
    """Every full-lattice mode with 0 < |n| < nbins*dn, its bin and |n| (by explicit loops
    over the integer components, each within |n_i| < nbins*dn, which every such mode
    satisfies; the bin test is b*dn <= |n| < (b+1)*dn)."""
    half = N // 2
    modes, bins = [], []
    kmax = nbins * dn
    kmax2 = kmax ** 2
    span = range(max(-half, -kmax + 1), min(half, kmax))
    for nx in span:
        for ny in span:
            for nz in span:
                q = nx * nx + ny * ny + nz * nz
                if q == 0 or q >= kmax2:
                    continue
                b = 0
                while ((b + 1) * dn) ** 2 <= q:
                    b += 1
                modes.append((nx, ny, nz))
                bins.append(b)
    return np.array(modes, dtype=np.int64).reshape(-1, 3), np.array(bins, dtype=np.int64)


def lattice_counts(N, dn, nbins):
    """Number of full-lattice modes in each bin (0 < |n| < nbins*dn, components in
    [-N/2, N/2)) without enumerating the lattice: with c1[q] the number of integers n,
    |n| < K = nbins*dn, with n^2 = q, the number of vectors with |n|^2 = q is the
    threefold convolution c1 * c1 * c1 at q (only q < K^2 is needed, so the component
    range never reaches -N/2)."""
    K = nbins * dn
    K2 = K * K
    c1 = np.zeros(K2, dtype=np.int64)
    c1[0] = 1
    j = np.arange(1, K)
    c1[j * j] = 2
    def conv(a):
        out = np.zeros(K2, dtype=np.int64)
        for v in range(K):
            q = v * v
            out[q:] += c1[q] * a[:K2 - q]
        return out
    c3 = conv(conv(c1))
    c3[0] = 0
    q = np.arange(K2)
    b = np.floor(np.sqrt(q)).astype(np.int64)
    b -= (b * b > q)
    b += ((b + 1) * (b + 1) <= q)
    return np.bincount(b // dn, weights=c3, minlength=nbins)[:nbins].astype(np.int64)


def amplitudes_direct(pos, wprime, box_min, L, N, assign, observer, los, modes, funcs,
                      method="interp", chunk=512):
    """Direct amplitudes A_f(n) = sum_p w'_p f(khat . rhat_p) Phi_p(n) for each f in funcs.

    method "interp": Phi is the interpolated phase of the assignment kernel;
    method "sumgal": Phi = exp(-2 pi i n . u_p / N) (no grid at all).
    Returns an array [len(funcs), len(modes)] of complex amplitudes.
    """
    pos = np.asarray(pos, np.float64)
    wprime = np.asarray(wprime, np.float64)
    u = (pos - np.asarray(box_min, np.float64)[None, :]) * (N / float(L))
    if los == 1:
        rh = np.zeros_like(pos)
        rh[:, 2] = 1.0
    else:
        d = pos - np.asarray(observer, np.float64)[None, :]
        rh = d / np.linalg.norm(d, axis=1)[:, None]
    modes = np.asarray(modes, np.int64)
    if method == "interp":
        # the phases of the frequencies (mod N) that the modes use, one column each
        freq = np.unique(modes % N)
        ph = [_axis_phase(u[:, i], N, assign, freq) for i in range(3)]
    out = np.zeros((len(funcs), len(modes)), dtype=np.complex128)
    for s in range(0, len(modes), chunk):
        m = modes[s:s + chunk]
        kh = m / np.linalg.norm(m, axis=1)[:, None]
        mu = rh @ kh.T                                   # [particles, modes]
        if method == "interp":
            idx = np.searchsorted(freq, m % N)
            phi = ph[0][:, idx[:, 0]] * ph[1][:, idx[:, 1]] * ph[2][:, idx[:, 2]]
        else:
            phi = np.exp(-2j * np.pi * (u @ m.T.astype(np.float64)) / N)
        wphi = wprime[:, None] * phi
        for j, f in enumerate(funcs):
            out[j, s:s + chunk] = np.sum(f(mu) * wphi, axis=0)
    return out


def direct_multipoles(gal_pos, gal_w, ran_pos, ran_w, gal_nbar, ran_nbar, *, N, box_min, L,
                      assign, observer=(0.0, 0.0, 0.0), los=0, compensate=2, dn=1, nbins=None,
                      norm_from=0, method="interp", chunk=512, ell_max=4):
    """P_ell per bin from direct amplitudes with Legendre polynomials evaluated per particle:

      P_ell(b) = (2 ell + 1) <Re[A_0 A_{L_ell}^*] / W^2>_b / I  -  delta_{ell 0} <N>_b / I.

    The catalogue scalars are recomputed here from their definitions (Sec. 2). Bins
    0 .. nbins-1 are evaluated (each bin's value depends only on its own modes, so the
    first bins of a large grid can be checked alone).
    """
    if nbins is None:
        nbins = N // (2 * dn)
    gw = np.asarray(gal_w, np.float64)
    rw = np.asarray(ran_w, np.float64)
    alpha = gw.sum() / rw.sum()
    if norm_from == 0:
        I = alpha * np.sum(rw ** 2 * np.asarray(ran_nbar, np.float64))
    else:
        I = np.sum(gw ** 2 * np.asarray(gal_nbar, np.float64))
    S = np.sum(gw ** 2) + alpha ** 2 * np.sum(rw ** 2)
    pos = np.concatenate([np.asarray(gal_pos, np.float64), np.asarray(ran_pos, np.float64)])
    wprime = np.concatenate([gw, -alpha * rw])
    modes, bins = lattice_modes(N, dn, nbins)
    ells = tuple(range(0, ell_max + 1, 2))
    funcs = [lambda mu, l=l: legendre(l, mu) for l in ells]
    A = amplitudes_direct(pos, wprime, box_min, L, N, assign, observer, los, modes, funcs, method, chunk)
    p = assign
    x = np.pi * modes / N
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(modes == 0, 1.0, np.sin(x) / np.where(modes == 0, 1.0, x))
    W2 = np.prod(sinc ** (2 * p), axis=1)
    s2 = np.sin(x) ** 2
    Cax = 1.0 - (2.0 / 3.0) * s2 if p == 2 else 1.0 - s2 + (2.0 / 15.0) * s2 * s2
    C = np.prod(Cax, axis=1)
    if compensate == 0:
        inv = np.ones(len(modes))
        noise = np.full(len(modes), S)
    elif compensate == 1:
        inv = 1.0 / W2
        noise = np.full(len(modes), S)
    else:
        inv = 1.0 / W2
        noise = S * C / W2
    cnt = np.bincount(bins, minlength=nbins)[:nbins]
    out = {"count": cnt, "alpha": alpha, "I": I, "S": S}
    ok = cnt > 0
    for j, l in enumerate(ells):
        q = np.real(A[0] * np.conj(A[j])) * inv
        s = np.bincount(bins, weights=q, minlength=nbins)[:nbins]
        val = (2 * l + 1) * s
        if l == 0:
            val = val - np.bincount(bins, weights=noise, minlength=nbins)[:nbins]
        out[l] = np.where(ok, val / (I * np.where(ok, cnt, 1)), 0.0)
    out["noise"] = np.where(ok, np.bincount(bins, weights=noise, minlength=nbins)[:nbins] /
                            (I * np.where(ok, cnt, 1)), 0.0)
    kn = np.linalg.norm(modes, axis=1)
    ks = np.bincount(bins, weights=kn, minlength=nbins)[:nbins]
    out["k_eff"] = np.where(ok, (2 * np.pi / L) * ks / np.where(ok, cnt, 1), 0.0)
    return out


def dft3_direct(grid):
    """Sum-grid: the 3D DFT of g[ix, iy, iz] by direct summation over all cells."""
    N = grid.shape[0]
    j = np.arange(N)
    E = np.exp(-2j * np.pi * np.outer(j, j) / N)      # E[n, j]
    # sum over each axis in turn; each contraction is a plain sum over cells
    t = np.einsum("ia,abc->ibc", E, grid)
    t = np.einsum("jb,ibc->ijc", E, t)
    return np.einsum("kc,ijc->ijk", E, t)


def wedges_direct(gal_pos, gal_w, ran_pos, ran_w, gal_nbar, ran_nbar, *, N, box_min, L, assign,
                  observer=(0.0, 0.0, 0.0), los=0, compensate=2, dn=1, nbins=None, norm_from=0, mu_split=0.5,
                  chunk=512):
    """Top-hat mu-wedges with each particle's own line of sight (Sec. 5, Eqs. 14 and 15,
    read as Yamamoto wedges: mu = k-hat . r-hat of the particle, as the sum over galaxies
    the paper compares with). With W_perp(mu) = 1[|mu| < mu_split] / mu_split and
    W_par(mu) = 1[|mu| >= mu_split] / (1 - mu_split) (each averages to 1 over directions),

      P_wedge(b) = <Re[A_0 A_W^*] / W^2>_b / I - <N>_b / I,    A_W(n) = sum_p w'_p W(mu_p) Phi_p(n),

    Phi the interpolated phase of the assignment kernel. Expanding W in Legendre
    polynomials gives P_wedge = sum_l <L_l>_wedge P_l over every even l; Eqs. (16)-(17) keep
    l <= 4. Returns {"perp", "par", "P0", "count"} per bin."""
    if nbins is None:
        nbins = N // (2 * dn)
    gw = np.asarray(gal_w, np.float64)
    rw = np.asarray(ran_w, np.float64)
    alpha = gw.sum() / rw.sum()
    I = alpha * np.sum(rw ** 2 * np.asarray(ran_nbar, np.float64)) if norm_from == 0 else \
        np.sum(gw ** 2 * np.asarray(gal_nbar, np.float64))
    S = np.sum(gw ** 2) + alpha ** 2 * np.sum(rw ** 2)
    pos = np.concatenate([np.asarray(gal_pos, np.float64), np.asarray(ran_pos, np.float64)])
    wprime = np.concatenate([gw, -alpha * rw])
    modes, bins = lattice_modes(N, dn, nbins)
    funcs = [lambda mu: np.ones_like(mu),
             lambda mu: (np.abs(mu) < mu_split) / mu_split,
             lambda mu: (np.abs(mu) >= mu_split) / (1.0 - mu_split)]
    A = amplitudes_direct(pos, wprime, box_min, L, N, assign, observer, los, modes, funcs, "interp", chunk)
    p = assign
    x = np.pi * modes / N
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(modes == 0, 1.0, np.sin(x) / np.where(modes == 0, 1.0, x))
    W2 = np.prod(sinc ** (2 * p), axis=1)
    s2 = np.sin(x) ** 2
    Cax = 1.0 - (2.0 / 3.0) * s2 if p == 2 else 1.0 - s2 + (2.0 / 15.0) * s2 * s2
    if compensate == 0:
        inv, noise = np.ones(len(modes)), np.full(len(modes), S)
    elif compensate == 1:
        inv, noise = 1.0 / W2, np.full(len(modes), S)
    else:
        inv, noise = 1.0 / W2, S * np.prod(Cax, axis=1) / W2
    cnt = np.bincount(bins, minlength=nbins)[:nbins]
    ok = cnt > 0
    den = I * np.where(ok, cnt, 1)
    nb = np.bincount(bins, weights=noise, minlength=nbins)[:nbins] / den
    out = {"count": cnt}
    for j, key in enumerate(("P0", "perp", "par")):
        q = np.bincount(bins, weights=np.real(A[0] * np.conj(A[j])) * inv, minlength=nbins)[:nbins]
        out[key] = np.where(ok, q / den - nb, 0.0)
    return out
