"""Small hand-built cases for the oracle pins (inputs only)."""
import math

import numpy as np

from paper_2603_21869_amd import cases as C


def box(n=(8, 8, 8), h=(0.1, 0.1, 0.1), dim=3, kinds=None, physics=0, nu=1e-3,
        alpha_T=1e-3, dt=1e-3, n_levels=1, solid=None, patches=None, **kw):
    nn = (n[0], n[1], n[2] if dim == 3 else 1)
    hh = (h[0], h[1], h[2] if dim == 3 else 1.0)
    if patches is None:
        patches = []
        if kinds is not None:
            for f in range(2 * dim):
                if kinds[f] is not None:
                    patches.append(C.Patch(f, *C._face_full(nn, f), kind=kinds[f]))
    fl = {k: np.zeros((nn[2], nn[1], nn[0])) for k in C.FIELDS}
    return C.Case(name="box", dim=dim, n=nn, h=hh, nu=nu, rho=1.0, alpha_T=alpha_T, dt=dt,
                  physics=physics, patches=patches, fields=fl, solid=solid, n_levels=n_levels, **kw)


def centres(case):
    nx, ny, nz = case.n
    hx, hy, hz = case.h
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * hz, (np.arange(ny) + 0.5) * hy,
                          (np.arange(nx) + 0.5) * hx, indexing="ij")
    return x, y, z
