"""Parity of the HIP path (through the C interface) with the FP64 oracle.

Bar: mode counts bit-exact; alpha, I, S to FP64 rounding; per multipole
e_l = max_b |P_l^GPU - P_l^oracle| / (P_0^oracle + <N>_b / I) <= 1e-5 (the raw shell
power is the scale FP32 rounding acts on); k_eff to 1e-6 relative.
"""
import numpy as np
import pytest

from conftest import x_row
from oracle import estimator as est
from paper_1505_05341_amd import catalogs

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1505_05341_amd as pk
    pk.load()
    return pk


def oracle_config(cfg):
    """The estimator's configuration (x_planes only sets how the GPU schedules its work)."""
    return est.Config(**{k: v for k, v in cfg.items() if k != "x_planes"})


def run_both(pk, gal, ran, cfg):
    print("case", {k: v for k, v in cfg.items() if k not in ("box_min", "observer")}, gal.n, ran.n, flush=True)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    got = pk.pk_multipoles(g, r, cfg)
    ref = est.pk_multipoles_streamed(gal.pos, gal.w, ran.pos, ran.w, oracle_config(cfg), gal.nbar, ran.nbar)
    return got, ref


def compare(got, ref, cfg, tol=TOL):
    np.testing.assert_array_equal(got["nmodes"], ref.nmodes)
    assert abs(got["alpha"] - ref.alpha) <= 1e-12 * abs(ref.alpha)
    assert abs(got["I"] - ref.I) <= 1e-12 * abs(ref.I)
    assert abs(got["S"] - ref.S) <= 1e-12 * abs(ref.S)
    ok = ref.nmodes > 0
    raw = np.abs(ref.P[0]) + ref.noise
    errs = {}
    for ell in range(0, cfg["ell_max"] + 1, 2):
        e = np.max(np.abs(got["P%d" % ell][ok] - ref.P[ell][ok]) / raw[ok])
        errs[ell] = e
    wperp, wpar = est.wedges(ref.P)
    errs["perp"] = np.max(np.abs(got["Pperp"][ok] - wperp[ok]) / raw[ok])
    errs["par"] = np.max(np.abs(got["Ppar"][ok] - wpar[ok]) / raw[ok])
    np.testing.assert_allclose(got["k_eff"][ok], ref.k_eff[ok], rtol=1e-6)
    np.testing.assert_allclose(got["noise"][ok], ref.noise[ok], rtol=1e-5)
    assert np.all(got["P0"][~ok] == 0)
    print("errors", errs, flush=True)
    for ell, e in errs.items():
        assert e <= tol, (ell, e)
    return errs


def test_tiny_plain_default(pk):
    gal, ran, cfg = catalogs.tiny_plain()
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


@pytest.mark.parametrize("kw", [
    dict(assign=3),
    dict(ell_max=2),
    dict(ell_max=0),
    dict(los=1),
    dict(compensate=0),
    dict(compensate=1, assign=3),
    dict(dn=3, nbins=5),
    dict(norm_from=1),
])
def test_tiny_plain_options(pk, kw):
    gal, ran, cfg = catalogs.tiny_plain(**kw)
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


@pytest.mark.parametrize("N,assign,dn,nbins", [(8, 2, 1, 4), (16, 3, 1, 8), (64, 2, 3, 10), (128, 3, 2, 31),
                                               (64, 3, 1, 32)])
def test_sizes_and_ragged_tiles(pk, N, assign, dn, nbins):
    """Several FFT sizes; nbins*dn not a multiple of the tile width (ragged last tile)."""
    L = 500.0
    box_min = (-250.0, -250.0, 600.0)
    gal = catalogs.uniform_box(3000, box_min, L, 11 + N, 3000 / L ** 3)
    ran = catalogs.uniform_box(30000, box_min, L, 12 + N, 3000 / L ** 3)
    cfg = catalogs.config_dict(N, box_min, L, assign=assign, dn=dn, nbins=nbins, observer=(10.0, -20.0, 5.0))
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


def test_small_clustered_mock(pk):
    """The clustered RSD recipe scaled down (N = 64, several tiles, strong clustering)."""
    gal, ran, cfg = catalogs.small_clustered(N=64, nbar=3e-4, ran_factor=10.0)
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


def test_small_clustered_tsc_dn2(pk):
    gal, ran, cfg = catalogs.small_clustered(N=128, nbar=1e-4, L=800.0, ran_factor=5.0, N_field=64,
                                             assign=3, dn=2)
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


def test_xgrid_rows_match_oracle(pk):
    """Stage check: sampled rows of all 22 x-transformed LOS-weighted grids (the 15 gathered
    and stored ones, and the 7 with a power of rhat_z of 2 or more as the combinations of
    stored rows that the identity sum_i rhat_i^2 = 1 gives, which the y pass forms)."""
    import torch
    gal, ran, cfg = catalogs.small_clustered(N=64, nbar=3e-4, ran_factor=10.0, assign=3)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    ws, layout = pk.stage_xgrids(g, r, cfg)
    c = est.Config(**cfg)
    alpha, I, S = est.catalogue_scalars(gal.w, ran.w, gal.nbar, ran.nbar)
    pos = np.concatenate([gal.pos, ran.pos]).astype(np.float64)
    wp = est.signed_weights(gal.w, ran.w, alpha)
    rng = np.random.default_rng(0)
    from paper_1505_05341_amd import native
    assert sorted(layout) == [m for m in range(22) if native.monomial(m)[2] <= 1]  # the 15 stored
    for m in range(22):
        mono = native.monomial(m)
        for _ in range(3):
            iy, iz = (int(v) for v in rng.integers(0, c.N, 2))
            ref = est.x_transformed_row(pos, wp, c, mono, iy, iz)
            # FP32 rounding scales with the sum of |terms| of the row (the row itself is a
            # density contrast, and grids such as rhat_x rhat_y change sign), which the
            # x-transformed |w'| row bounds at kx = 0 (|rhat^m| <= 1); a lost particle
            # would be ~1/1500 of it
            l1 = est.x_transformed_row(pos, np.abs(wp), c, (0, 0, 0), iy, iz)[0].real
            kx = layout[0][1]
            gotrow = x_row(pk, ws, layout, m, c.N, iz, iy)
            err = np.max(np.abs(gotrow - ref[:kx])) / l1
            assert err < 1e-5, (m, iy, iz, err)


@pytest.mark.parametrize("N,assign,los,kind,xs", [(32, 2, 0, "tiny", 0), (64, 3, 0, "clustered", 0),
                                                  (32, 2, 1, "tiny", 0), (64, 2, 0, "clustered", 0),
                                                  (64, 3, 0, "clustered", 8)])
def test_ell6_matches_oracle(pk, N, assign, los, kind, xs):
    """ell_max = 6: 50 monomial grids (28 gathered, 22 from the identity), 16 z-power
    groups, P6 from L_6; the whole estimator against the oracle (also in slabs of 8
    planes, and inside a batch next to an ell_max = 4 mock)."""
    if kind == "tiny":
        gal, ran, cfg = catalogs.tiny_plain(N=N, assign=assign, los=los, ell_max=6)
    else:
        gal, ran, cfg = catalogs.small_clustered(N=N, nbar=3e-4, ran_factor=10.0, assign=assign, los=los, ell_max=6)
    gcfg = dict(cfg, x_planes=xs) if xs else cfg
    got, ref = run_both(pk, gal, ran, gcfg)
    assert "P6" in got
    compare(got, ref, cfg)
    if kind == "clustered" and assign == 3:
        g = pk.DeviceCatalog.from_host(gal)
        r = pk.DeviceCatalog.from_host(ran)
        c4 = dict(cfg, ell_max=4)
        res, st = pk.pk_multipoles_batch([g, g, g], [r, r, r], [gcfg, c4, gcfg], lanes=2)
        assert st == [0, 0, 0] and "P6" in res[0] and "P6" not in res[1]
        compare(res[0], ref, cfg)
        compare(res[2], ref, cfg)
        np.testing.assert_array_equal(res[1]["nmodes"], ref.nmodes)


def test_ell6_xgrid_rows(pk):
    """All 50 x-transformed rows at ell_max = 6 (the degree-6 rows with a power of rhat_z
    of 2 or more come from up to 10 gathered rows each) against the oracle's rows."""
    from paper_1505_05341_amd import native
    gal, ran, cfg = catalogs.small_clustered(N=32, nbar=3e-4, ran_factor=10.0, assign=3, ell_max=6)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    ws, layout = pk.stage_xgrids(g, r, cfg)
    assert len(layout) == 28
    c = est.Config(**cfg)
    alpha, I, S = est.catalogue_scalars(gal.w, ran.w, gal.nbar, ran.nbar)
    pos = np.concatenate([gal.pos, ran.pos]).astype(np.float64)
    wp = est.signed_weights(gal.w, ran.w, alpha)
    rng = np.random.default_rng(6)
    iy, iz = (int(v) for v in rng.integers(0, c.N, 2))
    l1 = est.x_transformed_row(pos, np.abs(wp), c, (0, 0, 0), iy, iz)[0].real
    for m in range(50):
        kx = layout[0][1]
        ref = est.x_transformed_row(pos, wp, c, native.monomial(m), iy, iz)[:kx]
        err = np.max(np.abs(x_row(pk, ws, layout, m, c.N, iz, iy) - ref)) / l1
        assert err < 1e-5, (m, err)


def test_repeat_runs_agree(pk):
    gal, ran, cfg = catalogs.small_clustered(N=64, nbar=3e-4, ran_factor=10.0)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    a = pk.pk_multipoles(g, r, cfg)
    b = pk.pk_multipoles(g, r, cfg)
    np.testing.assert_array_equal(a["nmodes"], b["nmodes"])
    for ell in (0, 2, 4):
        raw = np.abs(a["P0"]) + a["noise"]
        ok = a["nmodes"] > 0
        # the assignment sums each cell in FP32 in an order set by atomics: runs agree to
        # the FP32 rounding of the cells (a few 1e-8 of the raw power per cell), amplified
        # by the P4 cancellation; measured at most 5e-7 over repeated runs on MI355X
        d = np.max(np.abs(a["P%d" % ell][ok] - b["P%d" % ell][ok]) / raw[ok])
        print("repeat runs: ell", ell, "max difference %.2e of the raw shell power" % d, flush=True)
        assert d < 2e-6


# ------------------------------------------------------------------------- error paths

def _errcase(pk, mutate_gal=None, mutate_ran=None, cfg_kw=None, expect=None, ws_bytes=None):
    import ctypes
    from paper_1505_05341_amd import native
    gal, ran, cfg = catalogs.tiny_plain(n_gal=200, n_ran=2000)
    if cfg_kw:
        cfg.update(cfg_kw)
    if mutate_gal:
        mutate_gal(gal)
    if mutate_ran:
        mutate_ran(ran)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    if ws_bytes is not None:
        import torch
        lib = native.load()
        c = native.make_config(cfg)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        res = native.PkResult()
        st = lib.pk_multipoles(ctypes.byref(c), ctypes.byref(g.c_struct()), ctypes.byref(r.c_struct()),
                               ctypes.c_void_p(ws.data_ptr()), ws_bytes, ctypes.byref(res), native.current_stream())
        assert st == expect
        return
    with pytest.raises(native.PkError) as ei:
        pk.pk_multipoles(g, r, cfg)
    assert ei.value.status == expect, str(ei.value)


def test_error_out_of_box(pk):
    def f(c):
        c.pos[5, 0] = 600.0
    _errcase(pk, mutate_gal=f, expect=-2)


def test_error_nan_position(pk):
    def f(c):
        c.pos[7, 1] = np.nan
    _errcase(pk, mutate_ran=f, expect=-3)


def test_error_nan_weight(pk):
    def f(c):
        c.w[3] = np.inf
    _errcase(pk, mutate_gal=f, expect=-3)


def test_error_particle_at_observer(pk):
    def f(c):
        c.pos[0] = (0.0, 0.0, 1500.0)
    # observer inside the box at a particle position
    _errcase(pk, mutate_gal=f, cfg_kw=dict(observer=(0.0, 0.0, 1500.0)), expect=-3)


def test_error_particle_at_float_observer(pk):
    """An observer that FP32 cannot hold exactly, with a particle at its FP32 rounding: the
    line of sight is zero in the arithmetic the assignment uses (the FP64 difference is
    not), so the call must fail with PK_EDOM instead of spreading a NaN through the bins."""
    obs = (0.1, 0.2, 1500.3)

    def f(c):
        c.pos[0] = np.array(obs, dtype=np.float32)
    _errcase(pk, mutate_gal=f, cfg_kw=dict(observer=obs), expect=-3)


def test_catalogue_shape_checks(pk):
    """The binding refuses arrays the kernels would read past the end of."""
    import torch
    from paper_1505_05341_amd import native
    pos = torch.zeros((10, 3), device="cuda")
    w = torch.ones(10, device="cuda")
    for bad in [(pos, w[:9]), (pos[:, :2].contiguous(), w), (pos, w, torch.ones(11, device="cuda")),
                (pos.to(torch.int32), w), (pos, w.to(torch.float64))]:
        with pytest.raises(ValueError):
            native.make_catalog(*bad)
    assert native.make_catalog(pos, w, w).n == 10


def test_error_bad_config(pk):
    _errcase(pk, cfg_kw=dict(N=48), expect=-6)
    _errcase(pk, cfg_kw=dict(ell_max=3), expect=-1)
    _errcase(pk, cfg_kw=dict(nbins=17), expect=-1)
    _errcase(pk, cfg_kw=dict(dn=0), expect=-1)


def test_error_workspace_too_small(pk):
    from paper_1505_05341_amd import native
    gal, ran, cfg = catalogs.tiny_plain(n_gal=200, n_ran=2000)
    need = native.workspace_size(cfg, gal.n, ran.n)
    _errcase(pk, expect=-4, ws_bytes=need - 256)


def test_error_zero_random_weight(pk):
    def f(c):
        c.w[:] = 0.0
    _errcase(pk, mutate_ran=f, expect=-3)


# ------------------------------------------------------------------------- batches

def test_batch_matches_single_calls_and_oracle(pk):
    """Uneven mocks of two size classes over two lanes; every mock equals its own single
    call and the oracle; a mock with an out-of-box particle reports PK_ERANGE alone."""
    mocks = []
    for i in range(7):
        N = 32 if i % 3 else 64
        L = 400.0 + 50 * i
        box_min = (-L / 2, -L / 2, 500.0)
        ng = 1500 + 700 * i
        gal = catalogs.uniform_box(ng, box_min, L, 100 + i, ng / L ** 3)
        ran = catalogs.uniform_box(10 * ng, box_min, L, 200 + i, ng / L ** 3)
        if i == 4:
            gal.pos[3, 2] = 499.0          # outside the box
        cfg = catalogs.config_dict(N, box_min, L, assign=2 if i % 2 else 3, dn=1)
        mocks.append((gal, ran, cfg))
    dg = [pk.DeviceCatalog.from_host(m[0]) for m in mocks]
    dr = [pk.DeviceCatalog.from_host(m[1]) for m in mocks]
    res, st = pk.pk_multipoles_batch(dg, dr, [m[2] for m in mocks], lanes=2)
    assert st[4] == -2 and res[4] is None
    for i, (gal, ran, cfg) in enumerate(mocks):
        if i == 4:
            continue
        assert st[i] == 0
        single = pk.pk_multipoles(dg[i], dr[i], cfg)
        np.testing.assert_array_equal(res[i]["nmodes"], single["nmodes"])
        raw = np.abs(single["P0"]) + single["noise"]
        ok = single["nmodes"] > 0
        for ell in (0, 2, 4):
            # the same kernels; only the FP32 cell-sum order differs (see the repeat-run
            # test); these mocks have 1,500-5,000 galaxies, so P4 cancels more: measured
            # at most 8.5e-7 on MI355X
            d = np.max(np.abs(res[i]["P%d" % ell][ok] - single["P%d" % ell][ok]) / raw[ok])
            print("batch vs single: mock", i, "ell", ell, "max difference %.2e" % d, flush=True)
            assert d < 4e-6
        if i in (0, 5):
            ref = est.pk_multipoles(gal.pos, gal.w, ran.pos, ran.w, est.Config(**cfg), gal.nbar, ran.nbar)
            compare(res[i], ref, cfg)


@pytest.mark.parametrize("N", [32, 128])
def test_every_schedule_matches_oracle(pk, N):
    """Both column-transform schedules of the y and z passes (16 or 8 values per thread)
    give the oracle's multipoles; the autotuner returns one of them and keeps it."""
    from paper_1505_05341_amd import native
    gal, ran, cfg = catalogs.small_clustered(N=N, nbar=3e-4, ran_factor=10.0, dn=1)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    ref = est.pk_multipoles_streamed(gal.pos, gal.w, ran.pos, ran.w, est.Config(**cfg), gal.nbar, ran.nbar)
    try:
        for ys in (16, 8):
            for zs in (16, 8):
                native.set_schedule(N, cfg["ell_max"], ys, zs)
                print("schedule", ys, zs, flush=True)
                compare(pk.pk_multipoles(g, r, cfg), ref, cfg)
        best = pk.autotune(g, r, cfg, reps=2)
        assert best[0] in (8, 16) and best[1] in (8, 16)
        assert native.get_schedule(N, cfg["ell_max"]) == best
        compare(pk.pk_multipoles(g, r, cfg), ref, cfg)
    finally:
        native.set_schedule(N, cfg["ell_max"], 8, 8)   # back to the defaults


@pytest.mark.parametrize("N,assign,xs", [(32, 2, 1), (32, 3, 4), (64, 3, 8), (64, 2, 32)])
def test_slabs_match_oracle(pk, N, assign, xs):
    """Out of core: the x and y transforms run slab by slab through a buffer of xs planes
    (as at N = 2048). The multipoles are the oracle's; the buffer holds the oracle's
    x-transformed rows of the first slab (z < xs, with the rows whose TSC stencil wraps to
    the top plane); a batch mixing slabbed and whole plans and the autotuner agree too."""
    from paper_1505_05341_amd import native
    gal, ran, cfg = catalogs.small_clustered(N=N, nbar=3e-4, ran_factor=10.0, assign=assign, dn=1)
    scfg = dict(cfg, x_planes=xs)
    assert native.x_planes(scfg, gal.n, ran.n) == xs
    got, ref = run_both(pk, gal, ran, scfg)
    compare(got, ref, cfg)
    g = pk.DeviceCatalog.from_host(gal)
    r = pk.DeviceCatalog.from_host(ran)
    ws, layout = pk.stage_xgrids(g, r, scfg)
    assert layout[0][2] == xs
    c = oracle_config(cfg)
    alpha, I, S = est.catalogue_scalars(gal.w, ran.w, gal.nbar, ran.nbar)
    pos = np.concatenate([gal.pos, ran.pos]).astype(np.float64)
    wp = est.signed_weights(gal.w, ran.w, alpha)
    rng = np.random.default_rng(N + xs)
    assert pk.xgrid_view(ws, layout, 0, N).shape[0] == xs
    for m in (0, 6, 21):   # 6 (rhat_z^2) and 21 (rhat_z^4) from the stored rows
        mono = native.monomial(m)
        for iz in sorted({0, xs - 1}):
            iy = int(rng.integers(0, N))
            ref_row = est.x_transformed_row(pos, wp, c, mono, iy, iz)
            kx = layout[0][1]
            gotrow = x_row(pk, ws, layout, m, N, iz, iy)
            scale = np.sqrt(np.mean(np.abs(ref_row[:kx]) ** 2)) + 1e-30
            assert np.max(np.abs(gotrow - ref_row[:kx])) / scale < 1e-5, (m, iy, iz)
    del ws
    res, st = pk.pk_multipoles_batch([g, g, g], [r, r, r], [scfg, cfg, scfg], lanes=2)
    assert st == [0, 0, 0]
    for out in res:
        compare(out, ref, cfg)
    if xs == 4:
        try:
            best = pk.autotune(g, r, scfg, reps=1)
            assert best[0] in (8, 16) and best[1] in (8, 16)
            compare(pk.pk_multipoles(g, r, scfg), ref, cfg)
        finally:
            native.set_schedule(N, cfg["ell_max"], 8, 8)   # back to the defaults


# ------------------------------------------------------------------------- degenerate inputs

def _grid_catalog(pos, w, nbar):
    return catalogs.Catalog(np.asarray(pos, np.float32), np.full(len(pos), w, np.float32),
                            np.full(len(pos), nbar, np.float32))


def test_particles_on_cell_edges_and_box_faces(pk):
    """Positions exactly on grid nodes (offset 0: all CIC weight on one cell, the TSC
    base cell rounds half up), on the lower box faces and one float32 step below the
    upper faces (the periodic wrap)."""
    N, L = 32, 320.0
    box_min = (-160.0, -160.0, 400.0)
    rng = np.random.default_rng(21)
    H = L / N
    nodes = np.asarray(box_min)[None, :] + rng.integers(0, N, (300, 3)) * H
    faces = np.asarray(box_min)[None, :] + rng.random((100, 3)) * L
    faces[:50, 0] = box_min[0]
    faces[50:, 2] = np.nextafter(np.float32(box_min[2] + L), np.float32(-np.inf))
    gal = _grid_catalog(np.concatenate([nodes, faces]), 1.0, 1e-4)
    ran = catalogs.uniform_box(4000, box_min, L, 22, 1e-4)
    for assign in (2, 3):
        cfg = catalogs.config_dict(N, box_min, L, assign=assign)
        got, ref = run_both(pk, gal, ran, cfg)
        compare(got, ref, cfg)


@pytest.mark.parametrize("assign", [2, 3])
def test_all_galaxies_in_one_cell(pk, assign):
    """Extreme clustering: every galaxy in one cell, so one grid row holds them all (many
    LDS chunks, one overloaded cell in the in-row sort and in the x pass's walk over the
    S base cells of a target cell), randoms uniform; CIC and TSC."""
    N, L = 64, 600.0
    box_min = (-300.0, -300.0, 700.0)
    rng = np.random.default_rng(31)
    H = L / N
    corner = np.asarray(box_min) + np.array([17, 40, 5]) * H
    gal = _grid_catalog(corner[None, :] + rng.random((6000, 3)) * H, 1.0, 1e-4)
    ran = catalogs.uniform_box(20000, box_min, L, 32, 1e-4)
    cfg = catalogs.config_dict(N, box_min, L, assign=assign)
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


def test_single_galaxy(pk):
    gal, ran, cfg = catalogs.tiny_plain(n_gal=1, n_ran=5000)
    got, ref = run_both(pk, gal, ran, cfg)
    compare(got, ref, cfg)


def test_empty_galaxy_catalogue_is_an_error(pk):
    """No galaxies: alpha = 0 and I = alpha sum_r w^2 nbar = 0, so the normalisation is
    undefined; reported as PK_EDOM."""
    def f(c):
        c.pos = c.pos[:0]
        c.w = c.w[:0]
        c.nbar = c.nbar[:0]
    _errcase(pk, mutate_gal=f, expect=-3)


def test_empty_batch(pk):
    res, st = pk.pk_multipoles_batch([], [], [])
    assert res == [] and st == []
