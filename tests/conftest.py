import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def gathered_weights(a, b, c):
    """Integer weights of the monomials with a power of rhat_z below 2 in rhat^(a,b,c),
    from rhat_z^2 = 1 - rhat_x^2 - rhat_y^2 applied until none of power 2 or more is left
    (the library stores only the x-transformed grids of those monomials)."""
    if c <= 1:
        return {(a, b, c): 1}
    out = {}
    for (da, db), s in (((0, 0), 1), ((2, 0), -1), ((0, 2), -1)):
        for k, v in gathered_weights(a + da, b + db, c - 2).items():
            out[k] = out.get(k, 0) + s * v
    return {k: v for k, v in out.items() if v}


def x_row(pk, ws, layout, m, N, iz, iy):
    """Row (iz, iy) of x-transformed grid m of the stage_xgrids workspace, complex128: the
    stored row, or for a monomial with a power of rhat_z of 2 or more the combination of
    stored rows that the identity gives."""
    from paper_1505_05341_amd import native
    index = {tuple(native.monomial(i)): i for i in layout}
    row = 0
    for mono, wgt in gathered_weights(*native.monomial(m)).items():
        r = pk.xgrid_row(ws, layout, index[mono], N, iz, iy).cpu().numpy().astype(np.float64)
        row = row + wgt * (r[:, 0] + 1j * r[:, 1])
    return row
