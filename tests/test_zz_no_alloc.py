"""The entry point that allocates nothing (pk_multipoles_noalloc), called through the C
interface, against pk_multipoles with a workspace on the same inputs: two calls in a row
on the shared scratch array, the second with smaller inputs (fewer particles, a smaller
grid, fewer bins), each to the parity bar of the estimator tests (mode counts exact,
alpha, I, S to FP64 rounding, e_l <= 1e-5 of the raw shell power); a configuration
larger than the array is refused with PK_EWORKSPACE and a message."""
import ctypes

import numpy as np
import pytest

from paper_1505_05341_amd import catalogs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1505_05341_amd import native
    lib = native.load()
    lib.pk_multipoles_noalloc.argtypes = [ctypes.POINTER(native.PkConfig), ctypes.POINTER(native.PkCatalog),
                                          ctypes.POINTER(native.PkCatalog), ctypes.POINTER(native.PkResult),
                                          ctypes.c_void_p]
    lib.pk_multipoles_noalloc.restype = ctypes.c_int32
    return lib


def _noalloc(lib, g, r, cfg):
    from paper_1505_05341_amd import api, native
    c = native.make_config(cfg)
    host = api._HostResult(c)
    res = native.PkResult()
    host.fill(res)
    st = lib.pk_multipoles_noalloc(ctypes.byref(c), ctypes.byref(g.c_struct()), ctypes.byref(r.c_struct()),
                                   ctypes.byref(res), native.current_stream())
    return st, (host.as_dict(res) if st == 0 else None)


def _compare(a, b, ell_max):
    np.testing.assert_array_equal(a["nmodes"], b["nmodes"])
    for key in ("alpha", "I", "S"):
        assert abs(a[key] - b[key]) <= 1e-12 * abs(b[key]), key
    ok = b["nmodes"] > 0
    raw = np.abs(b["P0"][ok]) + b["noise"][ok]
    errs = {ell: float(np.max(np.abs(a["P%d" % ell][ok] - b["P%d" % ell][ok]) / raw))
            for ell in range(0, ell_max + 1, 2)}
    print("noalloc vs workspace entry point", errs, flush=True)
    for ell, e in errs.items():
        assert e <= 1e-5, (ell, e)
    np.testing.assert_allclose(a["k_eff"][ok], b["k_eff"][ok], rtol=1e-12)


def test_noalloc_matches_workspace_entry_point(lib):
    import paper_1505_05341_amd as pk
    from paper_1505_05341_amd import native
    big = catalogs.small_clustered(N=64, nbar=3e-4, ran_factor=10.0, assign=3)
    small = catalogs.tiny_plain(n_gal=500, n_ran=5000, N=32, dn=2, nbins=8)
    for gal, ran, cfg in (big, small):
        need = native.workspace_size(cfg, gal.n, ran.n)
        print("case N=%d, %d + %d particles, needs %d bytes" % (cfg["N"], gal.n, ran.n, need), flush=True)
        assert need <= 64 << 20
        g = pk.DeviceCatalog.from_host(gal)
        r = pk.DeviceCatalog.from_host(ran)
        st, got = _noalloc(lib, g, r, cfg)
        assert st == 0, native.last_error()
        ref = pk.pk_multipoles(g, r, cfg)
        _compare(got, ref, cfg["ell_max"])


def test_noalloc_refuses_configurations_beyond_its_array(lib):
    import paper_1505_05341_amd as pk
    from paper_1505_05341_amd import native
    gal, ran, cfg = catalogs.tiny_plain(n_gal=500, n_ran=5000, N=32)
    cfg = dict(cfg, N=512, nbins=128)
    assert native.workspace_size(cfg, gal.n, ran.n) > 64 << 20
    st, _ = _noalloc(lib, pk.DeviceCatalog.from_host(gal), pk.DeviceCatalog.from_host(ran), cfg)
    assert st == -4
    assert "pk_multipoles_noalloc holds" in native.last_error()
