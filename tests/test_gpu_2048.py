"""Parity at N = 2048, the out-of-core size of the paper's timing table (Table 1): the
22 x-transformed grids would take 756 GB, so the x and y transforms run slab by slab
through a buffer of a few planes. The oracle cannot redo a 2048^3 estimator, so the
checks are those it can afford at any size:

* mode counts of every bin, bit-exact, against the lattice counts by convolution;
* the first bins (|n| < 6) of P_0, P_2, P_4, the wedges, k_eff and the noise against the
  interpolated-phase direct sum over particles (the gridded Yamamoto amplitudes mode by
  mode, Sec. 3: the FFT decomposition adds no approximation), on a survey-shaped catalogue
  in the paper's 3500 Mpc/h cube;
* a second run with another slab height agrees bin by bin at the repeat-run bar;
* rows of the x-transformed grids of the first slab against the oracle's rows (CIC and TSC,
  both blocks of a split row).
"""
import time

import numpy as np
import pytest

from conftest import x_row
from oracle import direct
from oracle import estimator as est
from paper_1505_05341_amd import catalogs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL = 1e-5
# row bound of the full-size tests (cells from FP64 coordinates, FP32 offsets, weights and
# sums: a few eps_32 per term relative to the row's sum of |terms|, at any N)
XTOL_2048 = 1e-5


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1505_05341_amd as pk
    pk.load()
    yield pk
    torch.cuda.empty_cache()


def _host(t):
    return t.cpu().numpy()


def test_survey_shell_2048(pk):
    import torch
    from paper_1505_05341_amd import native
    t = time.time()
    gal, ran, cfg = catalogs.survey_shell_device(N=2048, n_gal=20000, N_field=256)
    xs = native.x_planes(cfg, gal.n, ran.n)
    print("survey shell: %d galaxies + %d randoms, N = 2048, slab %d planes (%.1f s)"
          % (gal.n, ran.n, xs, time.time() - t), flush=True)
    assert xs < 2048
    ws = pk.Workspace()
    got = pk.pk_multipoles(gal, ran, cfg, workspace=ws)
    print("GPU run done", flush=True)
    counts = direct.lattice_counts(2048, cfg["dn"], cfg["nbins"])
    np.testing.assert_array_equal(got["nmodes"], counts)
    nchk = 3
    t = time.time()
    d = direct.direct_multipoles(_host(gal.pos), _host(gal.w), _host(ran.pos), _host(ran.w), _host(gal.nbar),
                                 _host(ran.nbar), N=2048, box_min=cfg["box_min"], L=cfg["L"],
                                 assign=cfg["assign"], observer=cfg["observer"], dn=cfg["dn"], nbins=nchk,
                                 chunk=32)
    print("oracle direct sum over %d modes: %.1f s" % (int(d["count"].sum()), time.time() - t), flush=True)
    np.testing.assert_array_equal(got["nmodes"][:nchk], d["count"])
    for key in ("alpha", "I", "S"):
        assert abs(got[key] - d[key]) <= 1e-12 * abs(d[key]), key
    np.testing.assert_allclose(got["k_eff"][:nchk], d["k_eff"], rtol=1e-6)
    np.testing.assert_allclose(got["noise"][:nchk], d["noise"], rtol=1e-5)
    raw = np.abs(d[0]) + d["noise"]
    wperp, wpar = est.wedges(d)
    errs = {ell: np.max(np.abs(got["P%d" % ell][:nchk] - d[ell]) / raw) for ell in (0, 2, 4)}
    errs["perp"] = np.max(np.abs(got["Pperp"][:nchk] - wperp) / raw)
    errs["par"] = np.max(np.abs(got["Ppar"][:nchk] - wpar) / raw)
    print("low-k errors", errs, flush=True)
    for k, e in errs.items():
        assert e <= TOL, (k, e)
    # another slab height: the same multipoles at the repeat-run bar, every bin
    other = pk.pk_multipoles(gal, ran, dict(cfg, x_planes=32), workspace=ws)
    ok = got["nmodes"] > 0
    raw_all = np.abs(got["P0"]) + got["noise"]
    for ell in (0, 2, 4):
        e = np.max(np.abs(other["P%d" % ell][ok] - got["P%d" % ell][ok]) / raw_all[ok])
        print("slab 32 vs %d, ell %d: %.2e" % (xs, ell, e), flush=True)
        assert e <= TOL, (ell, e)
    del ws


def _slab_catalogue(n, box_min, L, H, seed):
    """Uniform points in the first 20 planes and the top 2 planes of the box (so that the
    first slab's rows have particles, including those reached across the periodic wrap)."""
    rng = np.random.default_rng(seed)
    pos = np.asarray(box_min, np.float64)[None, :] + rng.random((n, 3)) * L
    zlo = box_min[2] + rng.random(n) * 20 * H
    zhi = box_min[2] + L - rng.random(n) * 2 * H
    pos[:, 2] = np.where(rng.random(n) < 0.8, zlo, zhi)
    nbar = np.full(n, 1e-4, np.float32)
    return catalogs.Catalog(catalogs._inside(pos, box_min, L), np.full(n, 0.5, np.float32), nbar)


@pytest.mark.parametrize("assign", [2, 3])
def test_first_slab_rows_2048(pk, assign):
    from paper_1505_05341_amd import native
    L, N = 3500.0, 2048
    box_min = (-1750.0, -1750.0, -450.0)
    H = L / N
    gal = _slab_catalogue(100000, box_min, L, H, 21 + assign)
    ran = _slab_catalogue(400000, box_min, L, H, 31 + assign)
    cfg = catalogs.config_dict(N, box_min, L, assign=assign, dn=2)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    ws, layout = pk.stage_xgrids(g, r, cfg)
    xs = layout[0][2]
    print("first slab: %d planes" % xs, flush=True)
    assert xs < N
    c = est.Config(**cfg)
    alpha, I, S = est.catalogue_scalars(gal.w, ran.w, gal.nbar, ran.nbar)
    pos = np.concatenate([gal.pos, ran.pos]).astype(np.float64)
    wp = est.signed_weights(gal.w, ran.w, alpha)
    rng = np.random.default_rng(5 + assign)
    for iz in sorted({0, 3, xs - 1}):
        iy = int(rng.integers(0, N))
        l1 = est.x_transformed_row(pos, np.abs(wp), c, (0, 0, 0), iy, iz)[0].real
        assert l1 > 0
        for m in (0, 6, 21):   # 6 and 21: combinations of stored rows
            kx = layout[0][1]
            row = x_row(pk, ws, layout, m, N, iz, iy)
            ref = est.x_transformed_row(pos, wp, c, native.monomial(m), iy, iz)[:kx]
            err = np.max(np.abs(row - ref)) / l1
            print("row", (iy, iz), "grid", m, "err %.2e" % err, flush=True)
            assert err < XTOL_2048, (iy, iz, m, err)
    del ws
