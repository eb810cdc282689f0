"""The synthetic lognormal RSD mocks that stand in for the paper's survey mocks (Sec. 4)
carry the clustering they are built with. The recipe draws a Gaussian field G with power
P_G (from xi_G = ln(1 + xi) of the target P), makes the galaxy field delta = e^(G - s^2/2) - 1
(power P, the target) and displaces each galaxy along its line of sight by f (Psi . rhat),
Psi from G / b. For a lognormal field the cross power of delta and G is exactly P_G (Stein's
lemma: <e^G G'> = xi_G <e^G>), so linear theory gives the redshift-space power
P(k) + 2 f mu^2 P_G(k) / b + f^2 mu^4 P_G(k) / b^2, i.e. with beta = f / b = 0.375

    P_0 = P + (2 beta / 3 + beta^2 / 5) P_G,  P_2 = (4 beta / 3 + 4 beta^2 / 7) P_G,
    P_4 = (8 beta^2 / 35) P_G,

the Kaiser multipoles when P_G = P. P and P_G are the generator's own spectra
(catalogs.lognormal_spectra), averaged over the field's modes in each bin. Measured by the
estimator, the mocks of both generators (numpy on the host, torch on the device) must give
these at 0.02 <= k < 0.06 h/Mpc.

Expected scatter: with the modes of a bin as independent Gaussian variables (the +-k
pairs counted once), Var(P_l) = (2l + 1)^2 <(P(mu) + N)^2 L_l(mu)^2>_mu / (N_k / 2), with
P(mu) the model above and N the shot noise; the bins are averaged. Allowed systematics:
the field is piecewise constant on its own grid (cells of 4.9 Mpc/h: a window suppressing
the power by <= 2% at k = 0.06), the displacement is linear in G, and positions wrap at the
faces of the periodic box: 4% on the monopole amplitude, 0.05 on P_2 / P_0 and 0.03 on
P_4 / P_0, plus 4 sigma.
"""
import numpy as np
import pytest

from paper_1505_05341_amd import catalogs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

BETA = 0.75 / 2.0
C0 = 2.0 * BETA / 3.0 + BETA ** 2 / 5.0
C2 = 4.0 * BETA / 3.0 + 4.0 * BETA ** 2 / 7.0
C4 = 8.0 * BETA ** 2 / 35.0
L_BOX = 2500.0
N_FIELD = 512


def _legendre(ell, mu):
    return {0: np.ones_like(mu), 2: 0.5 * (3 * mu ** 2 - 1), 4: (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8}[ell]


def binned_spectra(nbins, dn):
    """Mode averages of the generator's P and P_G in the estimator's bins (b dn <= |n| <
    (b + 1) dn, n in units of 2 pi / L), over the field's rfft half grid (the kz > 0 modes
    stand for their conjugates too)."""
    kmag, P, PG, _ = catalogs.lognormal_spectra(N_FIELD, L_BOX)
    n = kmag * L_BOX / (2.0 * np.pi)
    b = np.floor(n / dn + 1e-9).astype(np.int64)
    mult = np.full(kmag.shape, 2.0)
    mult[:, :, 0] = 1.0
    mult[:, :, -1] = 1.0
    sel = (b < nbins) & (kmag > 0)
    cnt = np.bincount(b[sel], weights=mult[sel], minlength=nbins)
    return (np.bincount(b[sel], weights=(mult * P)[sel], minlength=nbins) / np.maximum(cnt, 1),
            np.bincount(b[sel], weights=(mult * PG)[sel], minlength=nbins) / np.maximum(cnt, 1))


_spectra = {}


def check_kaiser(res, label, nbins, dn):
    if (nbins, dn) not in _spectra:
        _spectra[(nbins, dn)] = binned_spectra(nbins, dn)
    Pb, PGb = _spectra[(nbins, dn)]
    k = res["k_eff"]
    sel = (k >= 0.02) & (k < 0.06) & (res["nmodes"] > 0)
    assert sel.sum() >= 5
    mu = np.linspace(-1, 1, 2001)
    m0, m2, m4 = Pb + C0 * PGb, C2 * PGb, C4 * PGb
    var = {0: [], 2: [], 4: []}
    for b in np.nonzero(sel)[0]:
        Pmu = Pb[b] + (2 * BETA * mu ** 2 + BETA ** 2 * mu ** 4) * PGb[b] + res["noise"][b]
        for ell in (0, 2, 4):
            var[ell].append((2 * ell + 1) ** 2 * np.mean(Pmu ** 2 * _legendre(ell, mu) ** 2) / (res["nmodes"][b] / 2))
    var = {ell: np.asarray(v) for ell, v in var.items()}
    amp = res["P0"][sel] / m0[sel]
    amp_sig = np.sqrt(np.sum(var[0] / m0[sel] ** 2)) / sel.sum()
    s0 = np.sum(res["P0"][sel])
    r2, r4 = np.sum(res["P2"][sel]) / s0, np.sum(res["P4"][sel]) / s0
    e2, e4 = np.sum(m2[sel]) / np.sum(m0[sel]), np.sum(m4[sel]) / np.sum(m0[sel])
    r2_sig = np.sqrt(np.sum(var[2]) + r2 ** 2 * np.sum(var[0])) / s0
    r4_sig = np.sqrt(np.sum(var[4]) + r4 ** 2 * np.sum(var[0])) / s0
    print("%s: P0 / model = %.4f +- %.4f; P2/P0 = %.4f +- %.4f (model %.4f; Kaiser with P_G = P: %.4f); "
          "P4/P0 = %.4f +- %.4f (model %.4f); P_G / P = %.3f; %d bins"
          % (label, amp.mean(), amp_sig, r2, r2_sig, e2, C2 / (1 + C0), r4, r4_sig, e4,
             np.mean(PGb[sel] / Pb[sel]), sel.sum()), flush=True)
    assert abs(amp.mean() - 1.0) < 0.04 + 4 * amp_sig
    assert abs(r2 - e2) < 0.05 + 4 * r2_sig
    assert abs(r4 - e4) < 0.03 + 4 * r4_sig


def test_host_generator_kaiser_multipoles():
    import paper_1505_05341_amd as pk
    gal, ran, cfg = catalogs.clustered_rsd_512()
    res = pk.pk_multipoles(pk.DeviceCatalog.from_host(gal), pk.DeviceCatalog.from_host(ran), cfg)
    check_kaiser(res, "numpy generator, 512^3 field", cfg["nbins"], cfg["dn"])


def test_device_generator_kaiser_multipoles():
    import torch
    import paper_1505_05341_amd as pk
    gal, ran, box_min = catalogs.lognormal_rsd_device(N_field=N_FIELD, L=L_BOX, center=(0.0, 0.0, 2000.0),
                                                      nbar=3.0e-4, seed=12, ran_factor=20.0)
    cfg = catalogs.config_dict(512, box_min, L_BOX, assign=2, dn=2)
    res = pk.pk_multipoles(gal, ran, cfg)
    del gal, ran
    torch.cuda.empty_cache()
    check_kaiser(res, "torch generator, 512^3 field", cfg["nbins"], cfg["dn"])
