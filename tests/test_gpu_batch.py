"""Batched time steps of several grids (nfvm_step_batch): every grid ends
bitwise where nfvm_step on the grid alone ends, with the same per-step cycle
counts and statuses, whatever else is in the batch."""
import numpy as np
import pytest

from paper_2603_21869_amd import cases as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2603_21869_amd import nfvm
    nfvm.lib()
    return nfvm


def _mix():
    """Grids that take different paths through the batched iteration: mixed,
    FP32 and FP64 plans side by side; 2D and 3D; the LDS bottom solver (5
    levels) next to the coarsest-level solve (2 levels, and 1 level where it
    is level 0); no pre-smoothing
    (levels filled with zero); a tight cycle budget that stops early."""
    return [
        ("ch3d_mixed", C.channel3d(96, 32, 32, Lx=0.96, Ly=0.32, Lz=0.32, n_levels=5, n_steps=3,
                                   tol=1e-6, precision=C.PREC_MIXED, seed=21), {}),
        ("room_mixed", C.room3d(64, 32, 32, size=(1.28, 0.64, 0.64), vent=0.16,
                                side_range=(0.05, 0.3), clearance=0.1, seed=22, n_levels=5,
                                n_steps=3, precision=C.PREC_MIXED), {}),
        ("ch3d_mixed_2lev", C.channel3d(32, 16, 8, Lx=0.32, Ly=0.16, Lz=0.08, n_levels=2,
                                        n_steps=3, tol=1e-6, precision=C.PREC_MIXED, seed=23), {}),
        ("ch2d_mixed_1lev", C.channel2d(16, 16, L=1.0, H=1.0, n_levels=1, n_steps=3,
                                        precision=C.PREC_MIXED, seed=27), {}),
        ("ch2d_fp64", C.channel2d(128, 32, n_levels=4, n_steps=3, precision=C.PREC_FP64,
                                  seed=24), {}),
        ("ch3d_fp32_nu1_0", C.channel3d(64, 32, 32, Lx=0.64, Ly=0.32, Lz=0.32, n_levels=4,
                                        n_steps=3, tol=1e-5, precision=C.PREC_FP32,
                                        seed=25).copy(nu1=0), {}),
        ("ch3d_mixed_budget", C.channel3d(64, 32, 32, Lx=0.64, Ly=0.32, Lz=0.32, n_levels=5,
                                          n_steps=3, precision=C.PREC_MIXED, seed=26),
         dict(tol=1e-14, max_cycles=3)),
    ]


def _alone(nf, case, kw):
    g = nf.Grid(case, **kw)
    s, st = g.step(case.n_steps, allow=(0, nf.NFVM_E_NOTCONV))
    f = g.fields()
    g.close()
    return s, st, f


def test_batch_equals_alone(nf):
    mix = _mix()
    ref = [_alone(nf, c, kw) for _, c, kw in mix]
    grids = [nf.Grid(c, **kw) for _, c, kw in mix]
    n = mix[0][1].n_steps
    print(f"[batch] {len(grids)} grids, {n} steps", flush=True)
    s, sts, stats = nf.nfvm_step_batch([g.h for g in grids], n, allow=(0, nf.NFVM_E_NOTCONV))
    for (name, c, kw), g, (s1, st1, f1), s2, st2 in zip(mix, grids, ref, sts, stats):
        f2 = g.fields()
        print(f"   {name}: status {s1}/{s2} cycles {[x['cycles'] for x in st1]} "
              f"{[x['cycles'] for x in st2]}", flush=True)
        assert s2 == s1, name
        assert [x["cycles"] for x in st2] == [x["cycles"] for x in st1], name
        assert [x["status"] for x in st2] == [x["status"] for x in st1], name
        for a, b in zip(st1, st2):
            assert a["rel_residual"] == b["rel_residual"], name
            assert a["max_face_div"] == b["max_face_div"], name
            assert a["seconds"] > 0 and b["seconds"] > 0, name
        for k in f1:
            assert np.array_equal(f1[k], f2[k]), (name, k)
        g.close()
    assert s == nf.NFVM_E_NOTCONV  # the budget-limited grid


def test_batch_composition_does_not_matter(nf):
    """A grid stepped in two different batches (and in two calls) ends
    bitwise the same."""
    mix = _mix()
    (_, a, _), (_, b, _), (_, c, _) = mix[0], mix[1], mix[3]
    g1, g2 = nf.Grid(a), nf.Grid(b)
    nf.nfvm_step_batch([g1.h, g2.h], 2)
    nf.nfvm_step_batch([g2.h, g1.h], 1)
    h1, h3 = nf.Grid(a), nf.Grid(c)
    nf.nfvm_step_batch([h3.h, h1.h], 3)
    f1, f2 = g1.fields(), h1.fields()
    for k in f1:
        assert np.array_equal(f1[k], f2[k]), k
    for g in (g1, g2, h1, h3):
        g.close()


def test_batch_argument_errors(nf):
    c = _mix()[3][1]
    g = nf.Grid(c)
    with pytest.raises(nf.NfvmError) as e:
        nf.nfvm_step_batch([g.h, g.h], 1)
    assert e.value.status == nf.NFVM_E_INVAL
    s, sts, stats = nf.nfvm_step_batch([g.h], 0)
    assert s == nf.NFVM_OK and sts == [nf.NFVM_OK]
    g.close()


def test_batch_divergence_is_per_grid(nf):
    """A grid that diverges stops with NFVM_E_DIVERGED; the others in the
    batch finish as they would alone."""
    mix = _mix()
    good = mix[0][1]
    bad = mix[1][1].copy()
    bad.fields["u"][3, 4, 5] = np.nan
    s_ref, st_ref, f_ref = _alone(nf, good, {})
    gb, gg = nf.Grid(bad), nf.Grid(good)
    s, sts, stats = nf.nfvm_step_batch([gb.h, gg.h], good.n_steps,
                                       allow=(nf.NFVM_E_DIVERGED,))
    assert sts[0] == nf.NFVM_E_DIVERGED and sts[1] == nf.NFVM_OK
    f = gg.fields()
    for k in f:
        assert np.array_equal(f[k], f_ref[k]), k
    gb.close()
    gg.close()


def test_torch_caching_allocator_routes_grid_memory(nf):
    """With PyTorch's caching allocator installed (nfvm_set_allocator), a
    grid's device memory comes from it (torch's allocated bytes grow by the
    grid's footprint and fall back when the grid is freed), and the grid
    steps to bitwise the same fields as one on hipMalloc memory."""
    import torch
    case = C.channel3d(64, 16, 16, Lx=1.28, Ly=0.32, Lz=0.32, n_levels=3, n_steps=2)
    g = nf.Grid(case)
    g.step(2)
    ref = g.fields()
    g.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    nf.use_torch_allocator(True)
    try:
        g = nf.Grid(case)
        during = torch.cuda.memory_allocated()
        g.step(2)
        got = g.fields()
        g.close()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
    finally:
        nf.use_torch_allocator(False)
    fp = nf.nfvm_grid_footprint(nf.Desc(case))
    print(f"[alloc] torch bytes before={before} during={during} after={after} footprint={fp}",
          flush=True)
    assert during - before >= fp and after == before
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
