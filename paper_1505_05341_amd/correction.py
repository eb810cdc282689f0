"""Learned coarse-grid correction of the multipoles (the estimator's learned part).

A coarse grid is cheap but biased near its Nyquist frequency (aliasing of the signal,
imperfect window compensation); the fine-grid estimator is accurate but costs ~N^3 log N
more. The correction network (3 x 128 SiLU MLP, BF16 MFMA kernels in libpk) maps per-bin
features of a coarse-grid measurement to the fine-grid minus coarse-grid difference,
both measured by pk_multipoles itself on the same mocks:

  features  x = [k / k_Nyq, P0/R, P2/R, P4/R, noise/R, log10(nbar) + 3.5]
  targets   y = [(P0_f - P0_c)/R, (P2_f - P2_c)/R, (P4_f - P4_c)/R]

with R = P0_c + noise_c the raw coarse shell power of the bin. The corrected estimate is
P_l = P_l,c + R y_l. The plain fine-grid estimator remains the reference: the model is
judged against it on held-out mocks, and any catalogue outside the training domain
(nbar, box, grids) falls back to it.
"""
from __future__ import annotations

import json
import math

import numpy as np

from . import catalogs
from .api import Workspace, pk_multipoles

NFEAT = 6


def features(res, cfg, nbar):
    """Per-bin features of a coarse-grid result; rows for the non-empty bins only."""
    nb = cfg["nbins"]
    ok = res["nmodes"] > 0
    R = res["P0"] + res["noise"]
    kN = math.pi * cfg["N"] / cfg["L"]
    X = np.zeros((nb, NFEAT))
    X[:, 0] = res["k_eff"] / kN
    X[:, 1] = res["P0"] / np.where(ok, R, 1.0)
    X[:, 2] = res["P2"] / np.where(ok, R, 1.0)
    X[:, 3] = res["P4"] / np.where(ok, R, 1.0)
    X[:, 4] = res["noise"] / np.where(ok, R, 1.0)
    X[:, 5] = math.log10(nbar) + 3.5
    return X[ok], ok, R


def targets(res_c, res_f, ok, R):
    return np.stack([(res_f["P%d" % l][ok] - res_c["P%d" % l][ok]) / R[ok] for l in (0, 2, 4)], axis=1)


def coarse_fine_configs(box_min, L, N_coarse, N_fine, dn=1):
    """Same bins (in units of the fundamental mode) on both grids, up to the coarse Nyquist."""
    nb = N_coarse // (2 * dn)
    c = catalogs.config_dict(N_coarse, box_min, L, assign=2, dn=dn, nbins=nb)
    f = catalogs.config_dict(N_fine, box_min, L, assign=2, dn=dn, nbins=nb)
    return c, f


def make_pairs(n_mocks, seed0=5000, L=2500.0, center=(0.0, 0.0, 2000.0), N_coarse=256, N_fine=1024,
               N_field=512, nbar_range=(1e-4, 1e-3), ran_factor=10.0, log=None):
    """Method-generated training pairs: for each lognormal RSD mock (made on the GPU), the
    multipoles on the coarse and on the fine grid. Returns a dict of per-bin arrays."""
    import torch
    rng = np.random.default_rng(seed0)
    ws = Workspace()
    X, Y, meta = [], [], []
    for i in range(n_mocks):
        nbar = float(10 ** rng.uniform(math.log10(nbar_range[0]), math.log10(nbar_range[1])))
        gal, ran, box_min = catalogs.lognormal_rsd_device(N_field=N_field, L=L, center=center, nbar=nbar,
                                                          seed=seed0 + i, ran_factor=ran_factor)
        cc, cf = coarse_fine_configs(box_min, L, N_coarse, N_fine)
        rc = pk_multipoles(gal, ran, cc, ws)
        rf = pk_multipoles(gal, ran, cf, ws)
        x, ok, R = features(rc, cc, nbar)
        X.append(x)
        Y.append(targets(rc, rf, ok, R))
        for b in np.nonzero(ok)[0]:
            meta.append((i, b, nbar, R[b], rc["P0"][b], rc["P2"][b], rc["P4"][b], rf["P0"][b], rf["P2"][b],
                         rf["P4"][b], rc["k_eff"][b]))
        del gal, ran
        torch.cuda.empty_cache()
        if log and (i + 1) % max(1, n_mocks // 20) == 0:
            log("pairs: %d / %d mocks" % (i + 1, n_mocks))
    return {"X": np.concatenate(X), "Y": np.concatenate(Y), "meta": np.array(meta),
            "domain": {"nbar": list(nbar_range), "L": L, "N_coarse": N_coarse, "N_fine": N_fine}}


def _init_flat(din, dout, seed):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights, zero biases, canonical order."""
    rng = np.random.default_rng(seed)
    dims = [din, 128, 128, 128, dout]
    parts = []
    for i in range(4):
        lim = 1.0 / math.sqrt(dims[i])
        parts.append(rng.uniform(-lim, lim, dims[i] * dims[i + 1]))
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts).astype(np.float32)


class Correction:
    """The learned coarse-grid correction with its training domain and fine-grid fallback."""

    def __init__(self, seed=0):
        from .mlp import Mlp
        self.net = Mlp(NFEAT, 3)
        self.net.set_params(_init_flat(NFEAT, 3, seed))
        self.xm = np.zeros(NFEAT)
        self.xs = np.ones(NFEAT)
        self.ym = np.zeros(3)
        self.ys = np.ones(3)
        self.domain = None

    def fit(self, X, Y, domain, epochs=60, batch=2048, lr=2e-3, seed=0, log=None):
        import torch
        self.domain = dict(domain)
        self.xm, self.xs = X.mean(0), X.std(0) + 1e-12
        self.ym, self.ys = Y.mean(0), Y.std(0) + 1e-12
        xt = torch.tensor((X - self.xm) / self.xs, dtype=torch.float32, device="cuda")
        yt = torch.tensor((Y - self.ym) / self.ys, dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        n = xt.shape[0]
        hist = []
        steps = max(1, n // batch)
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g, device="cuda")
            lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))
            tot = 0.0
            for s in range(steps):
                idx = perm[s * batch:(s + 1) * batch]
                tot += float(self.net.train_step(xt[idx].contiguous(), yt[idx].contiguous(), lr_ep)[0])
            hist.append(tot / steps)
            if log and (ep + 1) % max(1, epochs // 10) == 0:
                log("epoch %d loss %.4g" % (ep + 1, hist[-1]))
        return hist

    def predict(self, X):
        import torch
        xt = torch.tensor((X - self.xm) / self.xs, dtype=torch.float32, device="cuda")
        return self.net.forward(xt).cpu().numpy().astype(np.float64) * self.ys + self.ym

    def in_domain(self, nbar, cfg_coarse):
        d = self.domain
        return (d is not None and d["nbar"][0] * 0.999 <= nbar <= d["nbar"][1] * 1.001
                and abs(cfg_coarse["L"] - d["L"]) < 1e-6 * d["L"] and cfg_coarse["N"] == d["N_coarse"])

    def corrected(self, res_c, cfg_c, nbar):
        """Corrected multipoles of a coarse-grid result, or None when the fallback applies."""
        if not self.in_domain(nbar, cfg_c):
            return None
        X, ok, R = features(res_c, cfg_c, nbar)
        y = self.predict(X)
        out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in res_c.items()}
        for j, l in enumerate((0, 2, 4)):
            out["P%d" % l][ok] = res_c["P%d" % l][ok] + R[ok] * y[:, j]
        return out

    def measure(self, gal, ran, box_min, nbar, ws=None):
        """Coarse grid + correction inside the training domain, plain fine grid outside it."""
        cc, cf = coarse_fine_configs(box_min, self.domain["L"], self.domain["N_coarse"], self.domain["N_fine"])
        cc["L"] = cf["L"] = float(self.domain["L"])
        rc = pk_multipoles(gal, ran, cc, ws)
        out = self.corrected(rc, cc, nbar)
        if out is None:
            return pk_multipoles(gal, ran, cf, ws), "fine"
        return out, "corrected"

    def save(self, path):
        np.savez(path, params=self.net.get_params(), xm=self.xm, xs=self.xs, ym=self.ym, ys=self.ys,
                 domain=json.dumps(self.domain))

    def load(self, path):
        z = np.load(path, allow_pickle=False)
        self.net.set_params(z["params"])
        self.xm, self.xs, self.ym, self.ys = z["xm"], z["xs"], z["ym"], z["ys"]
        self.domain = json.loads(str(z["domain"]))


def errors_vs_fine(meta, Yhat=None):
    """Mean and 90th-percentile |P_l - P_l,fine| / R over bins for the raw coarse estimate
    and (if Yhat is given) the corrected one. meta rows as built by make_pairs."""
    R = meta[:, 3]
    Pc = meta[:, 4:7]
    Pf = meta[:, 7:10]
    out = {}
    raw = np.abs(Pc - Pf) / R[:, None]
    out["raw_mean"] = raw.mean(0).tolist()
    out["raw_p90"] = np.percentile(raw, 90, axis=0).tolist()
    if Yhat is not None:
        cor = np.abs(Pc + R[:, None] * Yhat - Pf) / R[:, None]
        out["corrected_mean"] = cor.mean(0).tolist()
        out["corrected_p90"] = np.percentile(cor, 90, axis=0).tolist()
    return out
