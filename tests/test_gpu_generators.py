"""The synthetic lognormal RSD mocks that stand in for the paper's survey mocks (Sec. 4)
carry the clustering they are built with: measured by the estimator, their low-k
multipoles follow the input power law times the linear redshift-space (Kaiser) factors
for beta = f / b = 0.375: P_0 = (1 + 2 beta/3 + beta^2/5) P, P_2 = (4 beta/3 + 4 beta^2/7) P,
P_4 = (8 beta^2/35) P, i.e. P_2 / P_0 = 0.454 and P_4 / P_0 = 0.025. Both generators are
checked: the numpy one (host) and the torch one (device).

Expected scatter: with the modes of a bin as independent Gaussian variables (the +-k
pairs counted once), Var(P_l) = (2l + 1)^2 <(P(mu) + N)^2 L_l(mu)^2>_mu / (N_k / 2), with
P(mu) = (1 + beta mu^2)^2 P and N the shot noise; the bins of 0.02 <= k < 0.06 h/Mpc are
averaged. Allowed systematics: the field is piecewise constant on its own grid (cells of
4.9 Mpc/h: a window suppressing the power by <= 2% at k = 0.06), the displacement is linear
in the Gaussian field, and positions wrap at the faces of the periodic box: 4% on the
monopole amplitude, 0.05 on P_2 / P_0 and 0.03 on P_4 / P_0, plus 4 sigma.
"""
import numpy as np
import pytest

from paper_1505_05341_amd import catalogs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

BETA = 0.75 / 2.0
K0 = 1.0 + 2.0 * BETA / 3.0 + BETA ** 2 / 5.0
K2 = 4.0 * BETA / 3.0 + 4.0 * BETA ** 2 / 7.0
K4 = 8.0 * BETA ** 2 / 35.0


def p_in(k):
    return 2.0e4 * (k / 0.1) ** -1.5


def _legendre(ell, mu):
    return {0: np.ones_like(mu), 2: 0.5 * (3 * mu ** 2 - 1), 4: (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8}[ell]


def check_kaiser(res, label):
    k = res["k_eff"]
    sel = (k >= 0.02) & (k < 0.06) & (res["nmodes"] > 0)
    assert sel.sum() >= 5
    mu = np.linspace(-1, 1, 2001)
    ratios, sig = {}, {}
    # per-bin variances from the Kaiser model and the shot noise
    var = {0: [], 2: [], 4: []}
    for b in np.nonzero(sel)[0]:
        Pmu = (1 + BETA * mu ** 2) ** 2 * p_in(k[b]) + res["noise"][b]
        for ell in (0, 2, 4):
            var[ell].append((2 * ell + 1) ** 2 * np.mean(Pmu ** 2 * _legendre(ell, mu) ** 2) / (res["nmodes"][b] / 2))
    var = {ell: np.asarray(v) for ell, v in var.items()}
    amp = res["P0"][sel] / (K0 * p_in(k[sel]))
    amp_sig = np.sqrt(np.sum(var[0] / (K0 * p_in(k[sel])) ** 2)) / sel.sum()
    r2 = np.sum(res["P2"][sel]) / np.sum(res["P0"][sel])
    r4 = np.sum(res["P4"][sel]) / np.sum(res["P0"][sel])
    s0 = np.sum(res["P0"][sel])
    r2_sig = np.sqrt(np.sum(var[2]) + r2 ** 2 * np.sum(var[0])) / s0
    r4_sig = np.sqrt(np.sum(var[4]) + r4 ** 2 * np.sum(var[0])) / s0
    print("%s: P0 / (Kaiser P_in) = %.4f +- %.4f; P2/P0 = %.4f +- %.4f (expect %.4f); P4/P0 = %.4f +- %.4f "
          "(expect %.4f); %d bins" % (label, amp.mean(), amp_sig, r2, r2_sig, K2 / K0, r4, r4_sig, K4 / K0,
                                     sel.sum()), flush=True)
    assert abs(amp.mean() - 1.0) < 0.04 + 4 * amp_sig
    assert abs(r2 - K2 / K0) < 0.05 + 4 * r2_sig
    assert abs(r4 - K4 / K0) < 0.03 + 4 * r4_sig


def test_host_generator_kaiser_multipoles():
    import paper_1505_05341_amd as pk
    gal, ran, cfg = catalogs.clustered_rsd_512()
    res = pk.pk_multipoles(pk.DeviceCatalog.from_host(gal), pk.DeviceCatalog.from_host(ran), cfg)
    check_kaiser(res, "numpy generator, 512^3 field")


def test_device_generator_kaiser_multipoles():
    import torch
    import paper_1505_05341_amd as pk
    gal, ran, box_min = catalogs.lognormal_rsd_device(N_field=512, L=2500.0, center=(0.0, 0.0, 2000.0),
                                                      nbar=3.0e-4, seed=12, ran_factor=20.0)
    cfg = catalogs.config_dict(512, box_min, 2500.0, assign=2, dn=2)
    res = pk.pk_multipoles(gal, ran, cfg)
    del gal, ran
    torch.cuda.empty_cache()
    check_kaiser(res, "torch generator, 512^3 field")
