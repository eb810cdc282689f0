"""Seeded synthetic galaxy and random catalogues (inputs only; no estimator arithmetic).

These stand in for the survey mocks the paper measures (BOSS DR11 CMASS NGC
PTHalos mocks, about 525,000 galaxies with randoms at 10x their density, Sec. 4),
which are not available here. Both the HIP path and the FP64 oracle are fed
from this module; it holds none of the estimator's arithmetic.

Generators
----------
uniform_box       points uniform in a cube (the tiny plain-estimator case).
lognormal_rsd     a lognormal galaxy field with a power-law spectrum, Poisson
                  sampled, displaced along each particle's own line of sight by
                  the linear (Kaiser) redshift-space shift, plus uniform randoms
                  and FKP weights w = 1 / (1 + nbar P_FKP).

Every catalogue is float32 positions (n, 3), weights (n,) and nbar (n,), as the
C interface takes them. Configurations are plain dicts with the fields of the
estimator configuration.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np


@dataclass
class Catalog:
    pos: np.ndarray      # (n, 3) float32
    w: np.ndarray        # (n,) float32
    nbar: np.ndarray     # (n,) float32

    @property
    def n(self):
        return int(self.pos.shape[0])


def _inside(pos, box_min, L):
    """Round to float32 and keep every coordinate in [box_min, box_min + L)."""
    p = np.asarray(pos, dtype=np.float32)
    lo = np.asarray(box_min, dtype=np.float64)
    hi = lo + L
    for ax in range(3):
        col = p[:, ax]
        bad = col.astype(np.float64) >= hi[ax]
        if np.any(bad):
            col[bad] = np.nextafter(np.float32(hi[ax]), np.float32(-np.inf))
            # the float32 neighbour of the edge can itself round above it
            still = col.astype(np.float64) >= hi[ax]
            while np.any(still):
                col[still] = np.nextafter(col[still], np.float32(-np.inf))
                still = col.astype(np.float64) >= hi[ax]
        low = col.astype(np.float64) < lo[ax]
        while np.any(low):
            col[low] = np.nextafter(col[low], np.float32(np.inf))
            low = col.astype(np.float64) < lo[ax]
    return p


def uniform_box(n, box_min, L, seed, nbar, w=1.0):
    rng = np.random.default_rng(seed)
    pos = np.asarray(box_min, np.float64)[None, :] + rng.random((n, 3)) * L
    return Catalog(_inside(pos, box_min, L), np.full(n, w, np.float32), np.full(n, nbar, np.float32))


def config_dict(N, box_min, L, observer=(0.0, 0.0, 0.0), assign=2, ell_max=4, los=0,
                compensate=2, dn=1, nbins=0, norm_from=0):
    if nbins == 0:
        nbins = N // (2 * dn)
    return dict(N=int(N), box_min=tuple(float(v) for v in box_min), L=float(L),
                observer=tuple(float(v) for v in observer), assign=int(assign),
                ell_max=int(ell_max), los=int(los), compensate=int(compensate),
                dn=int(dn), nbins=int(nbins), norm_from=int(norm_from))


def tiny_plain(n_gal=2000, n_ran=20000, N=32, seed_gal=1505, seed_ran=5341, **cfg_kw):
    """Tiny plain case: observer at the origin, a 1000 Mpc/h cube centred at (0, 0, 1500),
    uniform galaxies and 10x uniform randoms, unit weights, CIC on 32^3, 16 linear bins
    up to the Nyquist frequency, ell = 0, 2, 4."""
    L = 1000.0
    box_min = (-500.0, -500.0, 1000.0)
    nbar = n_gal / L ** 3
    gal = uniform_box(n_gal, box_min, L, seed_gal, nbar)
    ran = uniform_box(n_ran, box_min, L, seed_ran, nbar)
    kw = dict(assign=2, ell_max=4, dn=1)
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, L, **kw)


def _fft_workers():
    return max(1, min(16, os.cpu_count() or 1))


def lognormal_spectra(N_field, L, amp=2.0e4, k0=0.1, slope=-1.5):
    """The spectra of the lognormal recipe on its field grid (rfft half grid, modes of the
    periodic box of side L): the target galaxy power P(k) = amp (k/k0)^slope (P(0) = 0),
    and the power P_G of the Gaussian field G with xi_G = ln(1 + xi) (negative values
    clipped, P_G(0) = 0). Returns (|k|, P, P_G, sigma_G^2), each (N, N, N/2 + 1)."""
    import scipy.fft as sfft

    N = int(N_field)
    H = L / N
    wk = _fft_workers()
    kx = 2.0 * np.pi * np.fft.fftfreq(N, d=H)
    kz = 2.0 * np.pi * np.fft.rfftfreq(N, d=H)
    kmag = np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        Pk = np.where(kmag > 0, amp * (kmag / k0) ** slope, 0.0)
    # xi(r) = (1/V) sum_k P(k) e^{ik.r}; irfftn carries 1/N^3
    xig = np.log1p(sfft.irfftn(Pk, s=(N, N, N), workers=wk) * (N ** 3 / L ** 3))
    PG = np.real(sfft.rfftn(xig, workers=wk)) * (L ** 3 / N ** 3)
    sigma2 = float(xig[0, 0, 0])
    del xig
    np.maximum(PG, 0.0, out=PG)
    PG[0, 0, 0] = 0.0
    return kmag, Pk, PG, sigma2


def lognormal_rsd(*, N_field, L, center, nbar, seed, amp=2.0e4, k0=0.1, slope=-1.5,
                  f=0.75, b=2.0, ran_factor=20.0, P_fkp=1.0e4, observer=(0.0, 0.0, 0.0)):
    """Lognormal RSD mock in a periodic cube of side L centred at `center`.

    Target galaxy power P(k) = amp (k/k0)^slope. Steps: xi from P on the grid;
    P_G from ln(1 + xi) (negative values clipped); a Gaussian field with P_G;
    delta = exp(G - sigma_G^2 / 2) - 1; Poisson counts nbar H^3 (1 + delta) with
    uniform positions inside each cell; displacement Psi(k) = i k G(k) / (b k^2)
    read at the galaxy's cell; s = x + f (Psi . rhat) rhat, wrapped into the box;
    uniform randoms (ran_factor times the galaxy count); w = 1 / (1 + nbar P_fkp).
    """
    import scipy.fft as sfft

    rng = np.random.default_rng(seed)
    N = int(N_field)
    H = L / N
    box_min = np.asarray(center, np.float64) - 0.5 * L
    wk = _fft_workers()
    kx = 2.0 * np.pi * np.fft.fftfreq(N, d=H)
    kz = 2.0 * np.pi * np.fft.rfftfreq(N, d=H)
    kmag, Pk, PG, sigma2 = lognormal_spectra(N, L, amp, k0, slope)
    del Pk
    k2 = kmag * kmag
    white = rng.standard_normal((N, N, N))
    Gk = sfft.rfftn(white, workers=wk)
    del white
    Gk *= np.sqrt(PG / H ** 3)
    del PG
    G = sfft.irfftn(Gk, s=(N, N, N), workers=wk)
    lam = nbar * H ** 3 * np.exp(G - 0.5 * sigma2)
    del G
    counts = rng.poisson(lam.ravel())
    del lam
    cells = np.repeat(np.arange(N ** 3, dtype=np.int64), counts)
    del counts
    ng = cells.size
    ijk = np.stack(np.unravel_index(cells, (N, N, N)), axis=1)
    x = box_min[None, :] + (ijk + rng.random((ng, 3))) * H
    # linear displacement from the Gaussian field's modes, Psi = i k G / (b k^2)
    with np.errstate(divide="ignore", invalid="ignore"):
        fac = np.where(k2 > 0, 1.0 / (b * k2), 0.0)
    disp = np.empty((ng, 3), np.float64)
    kvec = (kx[:, None, None], kx[None, :, None], kz[None, None, :])
    for ax in range(3):
        psi = sfft.irfftn(1j * kvec[ax] * fac * Gk, s=(N, N, N), workers=wk)
        disp[:, ax] = psi[ijk[:, 0], ijk[:, 1], ijk[:, 2]]
        del psi
    del Gk, fac, k2, kmag
    d = x - np.asarray(observer, np.float64)[None, :]
    rhat = d / np.linalg.norm(d, axis=1)[:, None]
    s = x + f * np.sum(disp * rhat, axis=1)[:, None] * rhat
    s = box_min[None, :] + np.mod(s - box_min[None, :], L)
    w = np.float32(1.0 / (1.0 + nbar * P_fkp))
    gal = Catalog(_inside(s, box_min, L), np.full(ng, w, np.float32), np.full(ng, nbar, np.float32))
    nr = int(round(ran_factor * ng))
    ran_pos = np.empty((nr, 3), np.float32)
    step = 1 << 24
    for s0 in range(0, nr, step):
        m = min(step, nr - s0)
        ran_pos[s0:s0 + m] = _inside(box_min[None, :] + rng.random((m, 3)) * L, box_min, L)
    ran = Catalog(ran_pos, np.full(nr, w, np.float32), np.full(nr, nbar, np.float32))
    return gal, ran, tuple(box_min)


def clustered_rsd_512(seed=2, N_field=512, N=512, **cfg_kw):
    """Clustered RSD mock: power law 2e4 (k/0.1)^-1.5 on 512^3, L = 2500 Mpc/h at 2000 Mpc/h,
    nbar = 3e-4 (about 4.7e6 galaxies), Kaiser f = 0.75, b = 2, 20x randoms, FKP P0 = 1e4,
    CIC on 512^3, ell = 0, 2, 4, bins of width 2 k_f."""
    gal, ran, box_min = lognormal_rsd(N_field=N_field, L=2500.0, center=(0.0, 0.0, 2000.0),
                                      nbar=3.0e-4, seed=seed)
    kw = dict(assign=2, ell_max=4, dn=2)
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, 2500.0, **kw)


def desi_scale_1024_device(seed=3, N_field=1024, N=1024, **cfg_kw):
    """DESI-scale single catalogue, made on the GPU: lognormal RSD mock (same power law,
    f = 0.75, b = 2) on a 1024^3 field, L = 4000 Mpc/h at 3000 Mpc/h, nbar = 4.6875e-4
    (about 3e7 galaxies), 20x randoms (about 6e8), FKP P0 = 1e4; TSC on 1024^3, all 22
    LOS-weighted grids (ell = 0, 2, 4), bins of width 2 k_f. Returns device catalogues."""
    gal, ran, box_min = lognormal_rsd_device(N_field=N_field, L=4000.0, center=(0.0, 0.0, 3000.0),
                                             nbar=3.0e7 / 4000.0 ** 3, seed=seed, ran_factor=20.0)
    kw = dict(assign=3, ell_max=4, dn=2)
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, 4000.0, **kw)


def small_clustered(N=64, seed=7, L=600.0, nbar=1.0e-3, ran_factor=10.0, N_field=None, **cfg_kw):
    """Scaled-down version of the clustered RSD mock (same recipe, small box) for parity tests."""
    gal, ran, box_min = lognormal_rsd(N_field=N_field or N, L=L, center=(0.0, 0.0, 1.2 * L),
                                      nbar=nbar, seed=seed, ran_factor=ran_factor)
    kw = dict(assign=2, ell_max=4, dn=1)
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, L, **kw)


# ---------------------------------------------------------------------------------
# Device generator (same recipe as lognormal_rsd, run with torch on the GPU). Input
# synthesis only: the estimator never calls it. Deterministic for a given seed on a
# given GPU model (torch's counter-based device generator).
# ---------------------------------------------------------------------------------

def lognormal_rsd_device(*, N_field, L, center, nbar, seed, amp=2.0e4, k0=0.1, slope=-1.5, f=0.75, b=2.0,
                         ran_factor=20.0, P_fkp=1.0e4, observer=(0.0, 0.0, 0.0), device="cuda"):
    """Lognormal RSD mock made on the GPU; returns (gal, ran, box_min) with gal and ran
    DeviceCatalog objects (float32 tensors on `device`)."""
    import torch
    from .api import DeviceCatalog

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    N = int(N_field)
    H = L / N
    f64 = torch.float64
    box_min = torch.tensor([c - 0.5 * L for c in center], dtype=f64, device=device)
    kx = 2.0 * np.pi * torch.fft.fftfreq(N, d=H, dtype=f64, device=device)
    kz = 2.0 * np.pi * torch.fft.rfftfreq(N, d=H, dtype=f64, device=device)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    kmag = torch.sqrt(k2)
    Pk = torch.where(kmag > 0, amp * (kmag.clamp_min(1e-30) / k0) ** slope, torch.zeros_like(kmag))
    xi = torch.fft.irfftn(Pk, s=(N, N, N)) * (N ** 3 / L ** 3)
    del Pk
    xig = torch.log1p(xi)
    del xi
    sigma2 = float(xig[0, 0, 0])
    PG = torch.fft.rfftn(xig).real * (L ** 3 / N ** 3)
    del xig
    PG.clamp_(min=0.0)
    PG[0, 0, 0] = 0.0
    white = torch.randn((N, N, N), generator=gen, dtype=f64, device=device)
    Gk = torch.fft.rfftn(white)
    del white
    Gk *= torch.sqrt(PG / H ** 3)
    del PG
    G = torch.fft.irfftn(Gk, s=(N, N, N))
    lam = nbar * H ** 3 * torch.exp(G - 0.5 * sigma2)
    del G
    counts = torch.poisson(lam.reshape(-1), generator=gen).to(torch.int64)
    del lam
    cells = torch.repeat_interleave(torch.arange(N ** 3, device=device), counts)
    del counts
    ng = int(cells.numel())
    ijk = torch.stack([cells // (N * N), (cells // N) % N, cells % N], dim=1)
    x = box_min[None, :] + (ijk.to(f64) + torch.rand((ng, 3), generator=gen, dtype=f64, device=device)) * H
    fac = torch.where(k2 > 0, 1.0 / (b * k2.clamp_min(1e-30)), torch.zeros_like(k2))
    kvec = (kx[:, None, None], kx[None, :, None], kz[None, None, :])
    disp = torch.empty((ng, 3), dtype=f64, device=device)
    for ax in range(3):
        psi = torch.fft.irfftn(1j * kvec[ax] * fac * Gk, s=(N, N, N))
        disp[:, ax] = psi[ijk[:, 0], ijk[:, 1], ijk[:, 2]]
        del psi
    del Gk, fac, k2, kmag, ijk, cells
    obs = torch.tensor(observer, dtype=f64, device=device)
    d = x - obs[None, :]
    rhat = d / torch.linalg.norm(d, dim=1, keepdim=True)
    s = x + f * torch.sum(disp * rhat, dim=1, keepdim=True) * rhat
    del d, rhat, disp, x
    s = box_min[None, :] + torch.remainder(s - box_min[None, :], L)
    w = float(np.float32(1.0 / (1.0 + nbar * P_fkp)))
    gpos = _inside_device(s, box_min, L)
    nr = int(round(ran_factor * ng))
    rpos = _inside_device(box_min[None, :] + torch.rand((nr, 3), generator=gen, dtype=f64, device=device) * L,
                          box_min, L)
    gal = DeviceCatalog(gpos, torch.full((ng,), w, dtype=torch.float32, device=device),
                        torch.full((ng,), nbar, dtype=torch.float32, device=device))
    ran = DeviceCatalog(rpos, torch.full((nr,), w, dtype=torch.float32, device=device),
                        torch.full((nr,), nbar, dtype=torch.float32, device=device))
    return gal, ran, tuple(float(v) for v in box_min.cpu().numpy())


def survey_shell_device(N=2048, seed=9, N_field=512, n_gal=525000, ran_factor=10.0, L=3500.0,
                        r_min=1200.0, r_max=1800.0, cap_deg=48.0, P_fkp=1.0e4, device="cuda", **cfg_kw):
    """Survey-shaped stand-in for the paper's timing catalogue (one CMASS-NGC-like mock of
    about 525,000 galaxies with randoms at 10x their density, in a cube of side 3500 Mpc/h,
    CIC, ell = 0, 2, 4; Sec. 4 and Table 1): a lognormal RSD field (same power law, f, b as
    the other mocks) on an N_field^3 grid, observed from the origin and cut to the shell
    r_min <= r < r_max inside a cap of half-angle cap_deg around +z (about 2.1 sr, the
    NGC area); nbar is set so that the shell holds about n_gal galaxies. Randoms are
    uniform in the same shell. The cube is centred at (0, 0, 1300), so the shell and the
    observer lie inside it. Returns (gal, ran, cfg) with device catalogues."""
    import torch
    from .api import DeviceCatalog

    cosc = float(np.cos(np.radians(cap_deg)))
    vol = 2.0 * np.pi * (1.0 - cosc) * (r_max ** 3 - r_min ** 3) / 3.0
    nbar = n_gal / vol
    center = (0.0, 0.0, 1300.0)
    gal_all, _, box_min = lognormal_rsd_device(N_field=N_field, L=L, center=center, nbar=nbar, seed=seed,
                                               ran_factor=0.0, P_fkp=P_fkp, device=device)

    def in_shell(p):
        p64 = p.to(torch.float64)
        r = torch.linalg.norm(p64, dim=1)
        return (r >= r_min) & (r < r_max) & (p64[:, 2] >= cosc * r)

    keep = in_shell(gal_all.pos)
    gpos = gal_all.pos[keep].contiguous()
    ng = int(gpos.shape[0])
    del gal_all
    # randoms: uniform in the shell's bounding box, kept inside the shell
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) + 1)
    nr = int(round(ran_factor * ng))
    half = r_max * float(np.sqrt(1.0 - cosc * cosc))
    lo = torch.tensor([-half, -half, r_min * cosc], dtype=torch.float64, device=device)
    ext = torch.tensor([2 * half, 2 * half, r_max - r_min * cosc], dtype=torch.float64, device=device)
    parts, have = [], 0
    while have < nr:
        q = lo[None, :] + torch.rand((max(nr - have, 1 << 20) * 3, 3), generator=gen, dtype=torch.float64,
                                     device=device) * ext[None, :]
        q32 = _inside_device(q, torch.tensor(box_min, dtype=torch.float64, device=device), L)
        q32 = q32[in_shell(q32)]
        parts.append(q32[:nr - have])
        have += int(parts[-1].shape[0])
    rpos = torch.cat(parts).contiguous()
    w = float(np.float32(1.0 / (1.0 + nbar * P_fkp)))
    f32 = torch.float32
    gal = DeviceCatalog(gpos, torch.full((ng,), w, dtype=f32, device=device),
                        torch.full((ng,), nbar, dtype=f32, device=device))
    ran = DeviceCatalog(rpos, torch.full((nr,), w, dtype=f32, device=device),
                        torch.full((nr,), nbar, dtype=f32, device=device))
    kw = dict(assign=2, ell_max=4, dn=2)
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, L, **kw)


def _inside_device(pos64, box_min, L):
    """float32 positions kept in [box_min, box_min + L) when compared in float64."""
    import torch
    p = pos64.to(torch.float32)
    lo = box_min[None, :]
    hi = lo + L
    for _ in range(4):
        over = p.to(torch.float64) >= hi
        if not bool(over.any()):
            break
        p = torch.where(over, torch.nextafter(p, torch.full_like(p, -np.inf)), p)
    for _ in range(4):
        under = p.to(torch.float64) < lo
        if not bool(under.any()):
            break
        p = torch.where(under, torch.nextafter(p, torch.full_like(p, np.inf)), p)
    return p.contiguous()


def device_catalog_to_host(cat):
    return Catalog(cat.pos.cpu().numpy(), cat.w.cpu().numpy(), cat.nbar.cpu().numpy())


# ---------------------------------------------------------------------------------
# Host-made catalogues for parity at the benchmark grids. Small enough for the FP64
# oracle, with the geometry and recipe of the benchmark workloads; the oracle's results
# for them are stored under tests/golden/ by a script that calls only the oracle.
# ---------------------------------------------------------------------------------

def desi_geometry_small(seed=31, nbar=3.0e-6, ran_factor=5.0, N=1024, **cfg_kw):
    """The DESI-scale geometry (L = 4000 Mpc/h centred at (0, 0, 3000), observer at the
    origin, lognormal RSD field with the same power law, f = 0.75, b = 2, FKP P0 = 1e4)
    at a low density: about 1.9e5 galaxies + 9.6e5 randoms, on the 1024^3 TSC plan of the
    benchmark (22 grids, bins of width 2 k_f up to the Nyquist frequency)."""
    gal, ran, box_min = lognormal_rsd(N_field=256, L=4000.0, center=(0.0, 0.0, 3000.0), nbar=nbar, seed=seed,
                                      ran_factor=ran_factor)
    kw = dict(assign=3, ell_max=4, dn=2)
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, 4000.0, **kw)


def clustered_geometry_small(seed=32, nbar=2.0e-5, ran_factor=5.0, N=512, **cfg_kw):
    """The clustered 512^3 geometry (L = 2500 Mpc/h centred at (0, 0, 2000), same recipe)
    at a low density: about 3.1e5 galaxies + 1.6e6 randoms, on the 512^3 CIC plan of the
    benchmark (bins of width 2 k_f), observed from an observer off the origin."""
    gal, ran, box_min = lognormal_rsd(N_field=256, L=2500.0, center=(0.0, 0.0, 2000.0), nbar=nbar, seed=seed,
                                      ran_factor=ran_factor)
    kw = dict(assign=2, ell_max=4, dn=2, observer=(120.0, -75.0, 40.0))
    kw.update(cfg_kw)
    return gal, ran, config_dict(N, box_min, 2500.0, **kw)


def checksum(gal, ran):
    """Counts and FP64 sums of the positions and weights: identifies a generated catalogue."""
    return {"n_gal": gal.n, "n_ran": ran.n,
            "pos_sum": [float(np.sum(c.pos[:, ax], dtype=np.float64)) for c in (gal, ran) for ax in range(3)],
            "w_sum": [float(np.sum(gal.w, dtype=np.float64)), float(np.sum(ran.w, dtype=np.float64))]}
