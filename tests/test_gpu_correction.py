"""The learned coarse-grid correction: trained on pairs the estimator itself measures
(coarse and fine grid on the same mocks), judged by the plain fine-grid estimator on
held-out mocks, and replaced by it outside the training domain (scaled-down sizes)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SMALL = dict(L=1000.0, center=(0.0, 0.0, 1500.0), N_coarse=32, N_fine=128, N_field=64,
             nbar_range=(3e-4, 3e-3), ran_factor=5.0)


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    from paper_1505_05341_amd import correction
    train = correction.make_pairs(48, seed0=100, **SMALL)
    test = correction.make_pairs(10, seed0=900, **SMALL)
    model = correction.Correction(seed=0)
    hist = model.fit(train["X"], train["Y"], train["domain"], epochs=150, batch=256, lr=3e-3)
    return correction, model, train, test, hist


def test_training_loss_falls(trained):
    _, _, _, _, hist = trained
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.5 * hist[0]


def test_correction_beats_raw_coarse_on_held_out_mocks(trained):
    correction, model, _, test, _ = trained
    err = correction.errors_vs_fine(test["meta"], model.predict(test["X"]))
    print("held-out |P - P_fine| / R:", err)
    # every multipole improves on average (the hexadecapole at least does not get worse)
    assert err["corrected_mean"][0] < 0.7 * err["raw_mean"][0]
    assert err["corrected_mean"][1] < err["raw_mean"][1]
    assert err["corrected_mean"][2] <= err["raw_mean"][2]


def test_out_of_domain_falls_back_to_fine_grid(trained):
    from paper_1505_05341_amd import catalogs
    import paper_1505_05341_amd as pk
    correction, model, _, _, _ = trained
    nbar = 1e-4                       # below the training range
    gal, ran, box_min = catalogs.lognormal_rsd_device(N_field=64, L=SMALL["L"], center=SMALL["center"],
                                                      nbar=nbar, seed=77, ran_factor=5.0)
    res, how = model.measure(gal, ran, box_min, nbar)
    assert how == "fine"
    _, cf = correction.coarse_fine_configs(box_min, SMALL["L"], SMALL["N_coarse"], SMALL["N_fine"])
    ref = pk.pk_multipoles(gal, ran, cf)
    for l in (0, 2, 4):
        np.testing.assert_allclose(res["P%d" % l], ref["P%d" % l], rtol=1e-6,
                                   atol=1e-6 * np.max(np.abs(ref["P0"]) + ref["noise"]))
    nbar_in = 1e-3
    gal, ran, box_min = catalogs.lognormal_rsd_device(N_field=64, L=SMALL["L"], center=SMALL["center"],
                                                      nbar=nbar_in, seed=78, ran_factor=5.0)
    _, how = model.measure(gal, ran, box_min, nbar_in)
    assert how == "corrected"
