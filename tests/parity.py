"""Shared helpers of the GPU parity tests: relative errors over fluid cells."""
import numpy as np

FIELDS = ("u", "v", "w", "p", "T", "k", "omega")


def fluid(case):
    return np.ones((case.n[2], case.n[1], case.n[0]), bool) if case.solid is None else case.solid == 0


def rel_err(a, b, mask, offset=0.0):
    """||a - b||_2 / ||b - offset||_2 over mask (offset: reference level, e.g. T_in)."""
    d = (a - b)[mask]
    den = np.linalg.norm((b - offset)[mask])
    num = np.linalg.norm(d)
    if den == 0.0:
        return num
    return num / den


def field_errors(case, gpu, ref):
    """Per-field relative errors plus 'vel', the velocity vector error relative
    to the velocity magnitude."""
    m = fluid(case)
    out = {}
    num = sum(np.sum(((gpu[c] - ref[c])[m]) ** 2) for c in ("u", "v", "w"))
    den = sum(np.sum((ref[c][m]) ** 2) for c in ("u", "v", "w"))
    out["vel"] = float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))
    for f in FIELDS:
        if f == "w" and case.dim == 2:
            continue
        off = case.T_ref if f == "T" else 0.0
        out[f] = rel_err(gpu[f], ref[f], m, off)
    return out
