"""Serving: continuous admission by HBM footprint, overlapping solves, and the
same result alone and in the mix."""
import time

import numpy as np
import pytest

from paper_2603_21869_amd import cases as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available()
    from paper_2603_21869_amd import nfvm
    nfvm.lib()
    return nfvm


def _requests():
    reqs = [
        C.channel3d(64, 32, 32, Lx=0.64, Ly=0.32, Lz=0.32, n_levels=5, n_steps=6, tol=1e-6,
                    precision=C.PREC_MIXED, seed=11),
        C.room3d(64, 32, 32, size=(1.28, 0.64, 0.64), vent=0.16, side_range=(0.05, 0.3),
                 clearance=0.1, seed=12, n_levels=5, n_steps=5, precision=C.PREC_MIXED),
        C.channel3d(96, 32, 32, Lx=0.96, Ly=0.32, Lz=0.32, n_levels=5, n_steps=4, tol=1e-6,
                    precision=C.PREC_MIXED, seed=13),
        C.channel2d(128, 32, n_levels=4, n_steps=8, precision=C.PREC_FP64, seed=14),
    ]
    return reqs


def test_alone_equals_in_mix(nf):
    """Each request served in a mix of concurrently running solves gives
    bitwise the fields it gives when run alone on a grid of its own."""
    reqs = _requests()
    alone = []
    for c in reqs:
        print(f"  alone: {c.name} prec={c.precision} steps={c.n_steps}",
              flush=True)
        g = nf.Grid(c)
        s, stats = g.step(c.n_steps, allow=(nf.NFVM_OK, nf.NFVM_E_DIVERGED, nf.NFVM_E_NOTCONV))
        why = nf.nfvm_last_error() if s != nf.NFVM_OK else ""
        out = g.fields()
        g.close()
        bad = [(i, st) for i, st in enumerate(stats) if st["status"] != nf.NFVM_OK]
        nonfinite = [k for k, v in out.items() if not np.isfinite(v).all()]
        assert s == nf.NFVM_OK, (c.name, s, why, bad[:1], stats, nonfinite)
        alone.append(out)
    srv = nf.nfvm_server_create(0.0, 3)
    tickets = []
    for c in reqs:
        d = nf.Desc(c)
        tickets.append((nf.nfvm_submit(srv, d, c.fields, c.n_steps), c))
    nf.nfvm_server_drain(srv)
    times = [nf.nfvm_request_times(srv, t) for t, _ in tickets]
    for (t, c), ref in zip(tickets, alone):
        s, out, st = nf.nfvm_poll(srv, t, (c.n[2], c.n[1], c.n[0]))
        assert s == nf.NFVM_OK
        for k in ref:
            assert np.array_equal(out[k], ref[k]), (c.name, k)
    nf.nfvm_server_destroy(srv)
    # at least two solves were resident at the same time
    spans = [(tm[1], tm[3]) for tm in times]
    overlap = any(a[0] < b[1] and b[0] < a[1] for i, a in enumerate(spans) for b in spans[i + 1:])
    assert overlap, spans


def test_admission_respects_budget(nf):
    """With a budget that holds one request at a time, requests run one after
    another; a request above the budget is refused at submit."""
    reqs = _requests()[:3]
    sizes = [nf.nfvm_grid_footprint(nf.Desc(c)) for c in reqs]
    budget = max(sizes) * 1.05
    srv = nf.nfvm_server_create(budget, 4)
    ts = [nf.nfvm_submit(srv, nf.Desc(c), c.fields, 2) for c in reqs]
    nf.nfvm_server_drain(srv)
    spans = sorted((nf.nfvm_request_times(srv, t)[1], nf.nfvm_request_times(srv, t)[3]) for t in ts)
    for a, b in zip(spans, spans[1:]):
        assert b[0] >= a[1] - 1e-6, spans
    for t, c in zip(ts, reqs):
        s, out, st = nf.nfvm_poll(srv, t, (c.n[2], c.n[1], c.n[0]))
        assert s == nf.NFVM_OK
    big = C.channel3d(128, 64, 64, n_levels=6)
    with pytest.raises(nf.NfvmError) as e:
        nf.nfvm_submit(srv, nf.Desc(big), big.fields, 1)
    assert e.value.status == nf.NFVM_E_NOMEM
    nf.nfvm_server_destroy(srv)


def test_failed_request_does_not_disturb_others(nf):
    reqs = _requests()[:2]
    bad = reqs[0].copy()
    bad.fields["u"][3, 4, 5] = np.inf
    srv = nf.nfvm_server_create(0.0, 2)
    tb = nf.nfvm_submit(srv, nf.Desc(bad), bad.fields, 2)
    tg = nf.nfvm_submit(srv, nf.Desc(reqs[1]), reqs[1].fields, 2)
    nf.nfvm_server_drain(srv)
    s, out, st = nf.nfvm_poll(srv, tb, (bad.n[2], bad.n[1], bad.n[0]), allow=(nf.NFVM_E_DIVERGED,))
    assert s == nf.NFVM_E_DIVERGED
    s, out, st = nf.nfvm_poll(srv, tg, (reqs[1].n[2], reqs[1].n[1], reqs[1].n[0]))
    assert s == nf.NFVM_OK and np.isfinite(out["u"]).all()
    nf.nfvm_server_destroy(srv)


def test_tune_fills_the_table(nf):
    """nfvm_tune records the tile choices of a shape before any grid of it is
    kept; a second call for the same shape adds nothing."""
    case = C.serve_case(dict(n=(64, 32, 32), geometry="channel", seed=3, n_steps=1))
    before = len(nf.nfvm_tuning_table())
    nf.nfvm_tune(nf.Desc(case))
    after = len(nf.nfvm_tuning_table())
    nf.nfvm_tune(nf.Desc(case))
    assert after >= before and len(nf.nfvm_tuning_table()) == after
    shapes = {(e[1], e[2], e[3]) for e in nf.nfvm_tuning_table()}
    assert (64, 32, 32) in shapes
