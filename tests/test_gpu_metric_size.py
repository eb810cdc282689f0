"""Parity at the benchmark grids, in the plans bench.py times, against stored FP64 oracle
results (tests/golden/oracle_<case>.json, written by tests/golden/make_oracle_goldens.py,
which calls only the oracle on the same seeded catalogue):

* the 1024^3 TSC plan of the DESI-scale workload (22 LOS-weighted grids, 256 bins of 2 k_f
  up to the Nyquist frequency, 8-column tiles, 1024-thread blocks), per-particle lines of
  sight: every bin, under each column-transform schedule of the y and z passes (16 or 8
  values per thread) -- the contraction of Sec. 3, Eqs. (10) and (12), with all its cross
  terms, at the size the accuracy target is stated on;
* the same catalogue and plan with the line of sight fixed to +z, against the
  one-transform plane-parallel form;
* the 512^3 CIC plan of the clustered workload, observer off the origin: every bin, each
  schedule;
* at 1024^3, sampled columns of the z-power groups H that pk_stage_fft leaves, against the
  oracle's transforms along x and y, and pk_stage_contract on them against the stored bins.

Bar (as the small parity tests): mode counts exact, alpha, I, S to FP64 rounding, k_eff to
1e-6, noise to 1e-5, e_l = max_b |P_l - P_l^oracle| / (P_0^oracle + <N>_b / I) <= 1e-5.
"""
import json
import os
import time

import numpy as np
import pytest

from oracle import estimator as est
from paper_1505_05341_amd import catalogs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

TOL = 1e-5
GOLD = os.path.join(os.path.dirname(__file__), "golden")
GEN = {"desi1024_tsc": catalogs.desi_geometry_small, "desi1024_tsc_los1": catalogs.desi_geometry_small,
       "clustered512_cic": catalogs.clustered_geometry_small}
SCHEDULES = [(16, 8), (8, 8), (16, 16), (8, 16)]


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1505_05341_amd as pk
    pk.load()
    yield pk
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def workspace(pk):
    ws = pk.Workspace()
    yield ws
    ws.buf = None


_cats = {}


def load_case(pk, case):
    """The stored oracle result and the device catalogue regenerated from its seed (checked
    against the stored checksum: counts exact, sums to 1e-9)."""
    with open(os.path.join(GOLD, "oracle_%s.json" % case)) as fh:
        gold = json.load(fh)
    cfg = gold["config"]
    cfg["box_min"], cfg["observer"] = tuple(cfg["box_min"]), tuple(cfg["observer"])
    key = GEN[case]
    if key not in _cats:
        _cats.clear()
        t = time.time()
        gal, ran, _ = key()
        chk = catalogs.checksum(gal, ran)
        print("%s: %d + %d particles regenerated (%.1f s)" % (case, gal.n, ran.n, time.time() - t), flush=True)
        _cats[key] = (gal, ran, pk.DeviceCatalog.from_host(gal), pk.DeviceCatalog.from_host(ran), chk)
    gal, ran, g, r, chk = _cats[key]
    ref = gold["catalogue"]
    assert (chk["n_gal"], chk["n_ran"]) == (ref["n_gal"], ref["n_ran"]), "the generator gave another catalogue"
    np.testing.assert_allclose(chk["pos_sum"] + chk["w_sum"], ref["pos_sum"] + ref["w_sum"], rtol=1e-9)
    return gold, cfg, gal, ran, g, r


def compare(got, gold, ell_max, tol=TOL):
    nm = np.asarray(gold["nmodes"])
    np.testing.assert_array_equal(got["nmodes"], nm)
    for key in ("alpha", "I", "S"):
        assert abs(got[key] - gold[key]) <= 1e-12 * abs(gold[key]), key
    ok = nm > 0
    P = {int(k): np.asarray(v) for k, v in gold["P"].items()}
    noise = np.asarray(gold["noise"])
    raw = np.abs(P[0]) + noise
    errs = {ell: float(np.max(np.abs(got["P%d" % ell][ok] - P[ell][ok]) / raw[ok])) for ell in range(0, ell_max + 1, 2)}
    wperp, wpar = est.wedges(P)
    errs["perp"] = float(np.max(np.abs(got["Pperp"][ok] - wperp[ok]) / raw[ok]))
    errs["par"] = float(np.max(np.abs(got["Ppar"][ok] - wpar[ok]) / raw[ok]))
    np.testing.assert_allclose(got["k_eff"][ok], np.asarray(gold["k_eff"])[ok], rtol=1e-6)
    np.testing.assert_allclose(got["noise"][ok], noise[ok], rtol=1e-5)
    print("e_l", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= tol, (k, e)
    return errs


@pytest.mark.parametrize("case", ["desi1024_tsc", "clustered512_cic"])
def test_every_bin_every_schedule(pk, workspace, case):
    from paper_1505_05341_amd import native
    gold, cfg, gal, ran, g, r = load_case(pk, case)
    N, ell = cfg["N"], cfg["ell_max"]
    before = native.get_schedule(N, ell)
    try:
        for ys, zs in SCHEDULES:
            native.set_schedule(N, ell, ys, zs)
            print("%s schedule (y, z) = (%d, %d)" % (case, ys, zs), flush=True)
            compare(pk.pk_multipoles(g, r, cfg, workspace), gold, ell)
    finally:
        native.set_schedule(N, ell, *before)


def test_plane_parallel_every_bin_1024(pk, workspace):
    gold, cfg, gal, ran, g, r = load_case(pk, "desi1024_tsc_los1")
    assert cfg["los"] == 1
    compare(pk.pk_multipoles(g, r, cfg, workspace), gold, cfg["ell_max"])


# Cells from FP64 coordinates (as the oracle takes them), FP32 offsets, weights, sums and
# transforms: a few eps_32 per term, relative to the sum of |terms| of the column
HTOL = 1e-5


def test_zgroup_columns_and_contract_1024(pk, workspace):
    """Columns of H_(n,c)(kx, ky, z) = sum_{a+b=n-c} c_abc tx^a ty^b Y_abc(kx, ky, z) for every
    z (t = 2 n / N), for the groups (0,0), (2,0), (4,1) and (4,4) (whose member r_z^4 is
    formed from the gathered monomials), at three (kx, ky), against the oracle's x-y
    transforms; then the contraction stage on that workspace against the stored bins."""
    from paper_1505_05341_amd import native
    gold, cfg, gal, ran, g, r = load_case(pk, "desi1024_tsc")
    N, ell = cfg["N"], cfg["ell_max"]
    ws = pk.stage_fft(g, r, cfg, workspace)
    c = est.Config(**cfg)
    alpha, I, S = est.catalogue_scalars(gal.w, ran.w, gal.nbar, ran.nbar)
    pos = np.concatenate([gal.pos, ran.pos]).astype(np.float64)
    wp = est.signed_weights(gal.w, ran.w, alpha)
    groups = {native.zgroup(ell, i): i for i in range(9)}
    coef = dict(((a, b, cc), w) for (a, b, cc), w in est.los_monomials(ell))
    for kx, ky in [(3, -7), (100, 41), (257, -300)]:
        kt = kx // 8
        l1 = est.xy_transformed_column(pos, np.abs(wp), c, (0, 0, 0), 0, 0).real
        for (n, zc) in [(0, 0), (2, 0), (4, 1), (4, 4)]:
            H, M = pk.hgrid_view(ws, cfg, gal.n, ran.n, groups[(n, zc)], kt)
            assert abs(ky) <= M
            got = H[:, ky + M, kx % 8].cpu().numpy()
            got = got[:, 0] + 1j * got[:, 1]
            ref = np.zeros(N, np.complex128)
            csum = 0
            for a in range(n - zc, -1, -1):
                b = n - zc - a
                w = coef[(a, b, zc)]
                csum += w
                ref += w * (2.0 * kx / N) ** a * (2.0 * ky / N) ** b * \
                    est.xy_transformed_column(pos, wp, c, (a, b, zc), kx, ky)
            err = np.max(np.abs(got - ref) / (csum * l1 + 1e-30))
            print("H group (%d,%d) at (kx, ky) = (%d, %d): err %.2e" % (n, zc, kx, ky, err), flush=True)
            assert err < HTOL, (n, zc, kx, ky, err)
    got = pk.stage_contract(ws, cfg, gal.n, ran.n)
    compare(got, gold, ell)
