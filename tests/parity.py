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


def field_max_errors(case, gpu, ref):
    """Per-field max-norm errors over fluid cells, max|a - b| / max|b - offset|
    ('vel': the largest velocity-vector difference over the largest speed),
    which an error confined to a few cells (a boundary row, a corner) cannot
    hide in."""
    m = fluid(case)
    out = {}
    du = np.sqrt(sum(((gpu[c] - ref[c])[m]) ** 2 for c in ("u", "v", "w")))
    sp = np.sqrt(sum((ref[c][m]) ** 2 for c in ("u", "v", "w")))
    out["vel"] = float(du.max() / sp.max()) if sp.max() > 0 else float(du.max())
    for f in FIELDS:
        if f == "w" and case.dim == 2:
            continue
        off = case.T_ref if f == "T" else 0.0
        d = np.abs((gpu[f] - ref[f])[m]).max()
        den = np.abs((ref[f] - off)[m]).max()
        out[f] = float(d / den) if den > 0 else float(d)
    return out


def check_fields(case, gpu, ref, bar, fields=("vel", "p", "k", "omega", "T"), floors=None,
                 tag=""):
    """Assert that both the relative L2 and the relative max-norm error of every
    listed field are within bar (a field in floors takes its own bar); T only
    when the case solves the energy equation.  Returns (l2, max) errors."""
    l2 = field_errors(case, gpu, ref)
    mx = field_max_errors(case, gpu, ref)
    use = [f for f in fields if f != "T" or case.physics & 2]
    print(f"   {tag} L2", {f: f"{l2[f]:.2e}" for f in use}, "max",
          {f: f"{mx[f]:.2e}" for f in use}, flush=True)
    for f in use:
        b = (floors or {}).get(f, bar)
        assert l2[f] <= b, (f, "L2", l2[f], b)
        assert mx[f] <= b, (f, "max", mx[f], b)
    return l2, mx
