"""Python front end of libpk: P_0, P_2, P_4 of device-resident catalogues.

    import torch, paper_1505_05341_amd as pk
    gal = pk.DeviceCatalog.from_host(gal_np)        # or pk.DeviceCatalog(pos, w, nbar)
    ran = pk.DeviceCatalog.from_host(ran_np)
    res = pk.pk_multipoles(gal, ran, cfg)            # cfg: dict of the C configuration fields

All arithmetic happens in the library's HIP kernels (include/pk.h); torch only holds
device memory and supplies the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import native


@dataclass
class DeviceCatalog:
    pos: "object"          # torch float32 (n, 3) on the GPU
    w: "object"            # torch float32 (n,)
    nbar: "object" = None  # torch float32 (n,) or None

    @property
    def n(self):
        return int(self.pos.shape[0])

    @staticmethod
    def from_host(cat, device="cuda"):
        import torch
        pos = torch.from_numpy(np.ascontiguousarray(cat.pos, dtype=np.float32)).to(device)
        w = torch.from_numpy(np.ascontiguousarray(cat.w, dtype=np.float32)).to(device)
        nbar = None
        if getattr(cat, "nbar", None) is not None:
            nbar = torch.from_numpy(np.ascontiguousarray(cat.nbar, dtype=np.float32)).to(device)
        return DeviceCatalog(pos, w, nbar)

    def c_struct(self):
        return native.make_catalog(self.pos, self.w, self.nbar)


class Workspace:
    """Reusable device workspace (a torch uint8 buffer), grown on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


class _HostResult:
    """Host arrays of one result and the pk_result struct that points at them."""

    def __init__(self, cfg):
        nb, nl = cfg.nbins, cfg.ell_max // 2 + 1
        self.cfg = cfg
        self.k, self.P, self.noise = np.zeros(nb), np.zeros(nb * nl), np.zeros(nb)
        self.nm, self.wedges = np.zeros(nb, dtype=np.int64), np.zeros(2 * nb)

    def fill(self, res):
        dp = ctypes.POINTER(ctypes.c_double)
        res.k_eff = self.k.ctypes.data_as(dp)
        res.P = self.P.ctypes.data_as(dp)
        res.noise = self.noise.ctypes.data_as(dp)
        res.nmodes = self.nm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        res.wedges = self.wedges.ctypes.data_as(dp)

    def as_dict(self, res):
        nb = self.cfg.nbins
        out = {"k_eff": self.k, "nmodes": self.nm, "noise": self.noise, "alpha": res.alpha, "I": res.I, "S": res.S,
               "Pperp": self.wedges[:nb].copy(), "Ppar": self.wedges[nb:].copy()}
        for j, ell in enumerate(range(0, self.cfg.ell_max + 1, 2)):
            out["P%d" % ell] = self.P[j * nb:(j + 1) * nb].copy()
        return out


def pk_multipoles(gal: DeviceCatalog, ran: DeviceCatalog, cfg: dict, workspace: Workspace | None = None,
                  stream=None):
    """Runs the estimator; returns k_eff, P0 [, P2, P4], the wedges Pperp and Ppar, noise,
    nmodes, alpha, I, S."""
    lib = native.load()
    c = native.make_config(cfg)
    cg, cr = gal.c_struct(), ran.c_struct()
    nbytes = native.workspace_size(cfg, gal.n, ran.n)
    ws = (workspace or Workspace()).get(nbytes)
    host = _HostResult(c)
    res = native.PkResult()
    host.fill(res)
    s = stream if stream is not None else native.current_stream()
    native.check(lib.pk_multipoles(ctypes.byref(c), ctypes.byref(cg), ctypes.byref(cr),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(res), s))
    return host.as_dict(res)


def pk_multipoles_batch(gals, rans, cfgs, lanes: int = 2, workspace: Workspace | None = None, stream=None):
    """Batched estimator over lists of device catalogues and configurations.

    Returns (results, statuses): one result dict per mock (None where its status is not
    PK_OK) and the per-mock status codes."""
    lib = native.load()
    n = len(cfgs)
    if not (len(gals) == len(rans) == n):
        raise ValueError("gals, rans and cfgs must have the same length")
    CfgArr = native.PkConfig * max(n, 1)
    CatArr = native.PkCatalog * max(n, 1)
    carr = CfgArr(*[native.make_config(c) for c in cfgs])
    garr = CatArr(*[g.c_struct() for g in gals])
    rarr = CatArr(*[r.c_struct() for r in rans])
    nbytes = ctypes.c_size_t()
    native.check(lib.pk_workspace_size_batch(carr, garr, rarr, n, lanes, ctypes.byref(nbytes)))
    ws = (workspace or Workspace()).get(int(nbytes.value))
    outs = (native.PkResult * max(n, 1))()
    keep = []
    for i in range(n):
        keep.append(_HostResult(carr[i]))
        keep[i].fill(outs[i])
    status = (ctypes.c_int32 * max(n, 1))()
    s = stream if stream is not None else native.current_stream()
    native.check(lib.pk_multipoles_batch(carr, garr, rarr, n, lanes, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         outs, status, s))
    results = []
    for i in range(n):
        if status[i] != native.PK_OK:
            results.append(None)
            continue
        results.append(keep[i].as_dict(outs[i]))
    return results, [int(status[i]) for i in range(n)]


def stage_xgrids(gal: DeviceCatalog, ran: DeviceCatalog, cfg: dict, workspace: Workspace | None = None):
    """Runs up to the fused assignment + x transform of the first slab of planes and
    returns (workspace tensor, layout), layout[m] = (byte offset, kx_count, planes, tile
    width W) of grid m (complex64 X[z][kx / W][y][kx % W] for z < planes; see xgrid_view)
    for every stored grid: the monomials with a power of rhat_z below 2 (the others follow
    from them, rhat_z^2 = 1 - rhat_x^2 - rhat_y^2)."""
    import torch
    lib = native.load()
    c = native.make_config(cfg)
    nbytes = native.workspace_size(cfg, gal.n, ran.n)
    ws = (workspace or Workspace()).get(nbytes)
    native.check(lib.pk_stage_xgrids(ctypes.byref(c), ctypes.byref(gal.c_struct()), ctypes.byref(ran.c_struct()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), native.current_stream()))
    torch.cuda.synchronize()
    layout = {}
    planes = native.x_planes(cfg, gal.n, ran.n)
    hoff, hm, width = ctypes.c_size_t(), ctypes.c_int32(), ctypes.c_int32()
    native.check(lib.pk_hgrid_layout(ctypes.byref(c), gal.n, ran.n, 0, 0, ctypes.byref(hoff), ctypes.byref(hm),
                                     ctypes.byref(width)))
    for m in range(native.num_grids(c.ell_max)):
        if native.monomial(m)[2] > 1:
            continue
        off = ctypes.c_size_t()
        kx = ctypes.c_int32()
        native.check(lib.pk_xgrid_layout(ctypes.byref(c), gal.n, ran.n, m, ctypes.byref(off), ctypes.byref(kx)))
        layout[m] = (int(off.value), int(kx.value), planes, int(width.value))
    return ws, layout


def stage_fft(gal: DeviceCatalog, ran: DeviceCatalog, cfg: dict, workspace: Workspace | None = None):
    """Runs up to the transforms along y of every slab and returns the workspace tensor,
    which then holds the z-power groups H (see hgrid_view)."""
    import torch
    lib = native.load()
    c = native.make_config(cfg)
    nbytes = native.workspace_size(cfg, gal.n, ran.n)
    ws = (workspace or Workspace()).get(nbytes)
    native.check(lib.pk_stage_fft(ctypes.byref(c), ctypes.byref(gal.c_struct()), ctypes.byref(ran.c_struct()),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), native.current_stream()))
    torch.cuda.synchronize()
    return ws


def hgrid_view(ws, cfg: dict, n_gal: int, n_ran: int, group: int, kx_tile: int):
    """complex64 H[z][ky + M][column] of one z-power group and kx tile in the workspace left by
    stage_fft, as (N, 2 M + 1, tile columns, 2) float32, and M."""
    import torch
    lib = native.load()
    c = native.make_config(cfg)
    off, M, tk = ctypes.c_size_t(), ctypes.c_int32(), ctypes.c_int32()
    native.check(lib.pk_hgrid_layout(ctypes.byref(c), n_gal, n_ran, group, kx_tile, ctypes.byref(off),
                                     ctypes.byref(M), ctypes.byref(tk)))
    N, M, tk, off = c.N, int(M.value), int(tk.value), int(off.value)
    nbytes = N * (2 * M + 1) * tk * 8
    return ws[off:off + nbytes].view(torch.float32).view(N, 2 * M + 1, tk, 2), M


def stage_contract(ws, cfg: dict, n_gal: int, n_ran: int):
    """The z transform, contraction, binning and finalisation on the workspace left by
    stage_fft; returns the same dictionary as pk_multipoles."""
    lib = native.load()
    c = native.make_config(cfg)
    host = _HostResult(c)
    res = native.PkResult()
    host.fill(res)
    native.check(lib.pk_stage_contract(ctypes.byref(c), n_gal, n_ran, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       ctypes.byref(res), native.current_stream()))
    return host.as_dict(res)


def xgrid_view(ws, layout, m, N):
    """complex64 values X[z][y][kx] (z < the slab height) of grid m inside the workspace
    returned by stage_xgrids, as (planes, N, kx, 2) float32: a strided view of the
    library's tile-major storage ([z][kx / W][y][kx % W], W = the tile width)."""
    import torch
    off, kx, planes, w = layout[m]
    nbytes = planes * N * kx * 8
    raw = ws[off:off + nbytes].view(torch.float32)
    return raw.view(planes, kx // w, N, w, 2).permute(0, 2, 1, 3, 4).reshape(planes, N, kx, 2)


def xgrid_row(ws, layout, m, N, z, y):
    """Row (z, y) of grid m of the stage_xgrids workspace as (kx, 2) float32 (a copy of
    that row only: xgrid_view reorders the whole tile-major grid)."""
    import torch
    off, kx, planes, w = layout[m]
    raw = ws[off:off + planes * N * kx * 8].view(torch.float32)
    return raw.view(planes, kx // w, N, w, 2)[z, :, y].reshape(kx, 2)


def autotune(gal: DeviceCatalog, ran: DeviceCatalog, cfg: dict, reps: int = 3, workspace: Workspace | None = None):
    """Times both column-transform schedules of the y and z passes on these inputs, keeps
    the fastest for (N, ell_max) in the library's table and returns (y_values, z_values)."""
    lib = native.load()
    c = native.make_config(cfg)
    nbytes = native.workspace_size(cfg, gal.n, ran.n)
    ws = (workspace or Workspace()).get(nbytes)
    y, z = ctypes.c_int32(), ctypes.c_int32()
    native.check(lib.pk_autotune(ctypes.byref(c), ctypes.byref(gal.c_struct()), ctypes.byref(ran.c_struct()),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), int(reps), ctypes.byref(y),
                                 ctypes.byref(z), native.current_stream()))
    return int(y.value), int(z.value)
