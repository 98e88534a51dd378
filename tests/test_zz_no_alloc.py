"""nfvm_mg_solve_device_noalloc (the pressure solve with library-held
scratch, for callers that cannot allocate) against nfvm_mg_solve_device on
the same device inputs: two calls in a row, the second on a smaller grid, each
bitwise equal to the allocating entry point (same kernels, same order)."""
import numpy as np
import pytest

from paper_2603_21869_amd import cases as C
from tests.parity import fluid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2603_21869_amd import nfvm
    nfvm.lib()
    return nfvm


def _solve_both(nf, case, seed, forced=-1):
    import torch
    g = nf.Grid(case)
    m = fluid(case)
    b = np.random.default_rng(seed).standard_normal(g.shape) * m
    bd = torch.from_numpy(b).cuda()
    xa = torch.zeros_like(bd)
    xb = torch.zeros_like(bd)
    torch.cuda.synchronize()
    sa, _ = nf.nfvm_mg_solve_device(g.h, bd.data_ptr(), xa.data_ptr(), tol=1e-8, max_cycles=80,
                                    forced_cycles=forced)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sb, _ = nf.nfvm_mg_solve_device_noalloc(g.h, bd.data_ptr(), xb.data_ptr(), tol=1e-8,
                                            max_cycles=80, forced_cycles=forced)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    g.close()
    return sa, sb, xa.cpu().numpy(), xb.cpu().numpy(), free0, free1


def test_noalloc_solve_equals_allocating_solve(nf):
    big = C.room3d(128, 64, 32, size=(10.0, 4.0, 3.0), seed=3, n_levels=5,
                   precision=C.PREC_MIXED)
    small = C.channel3d(64, 16, 16, Lx=1.28, Ly=0.32, Lz=0.32, n_levels=3,
                        precision=C.PREC_FP64)
    for i, (case, seed) in enumerate(((big, 1), (small, 2))):
        print(f"   noalloc: {case.name} prec={case.precision}", flush=True)
        sa, sb, xa, xb, free0, free1 = _solve_both(nf, case, seed)
        print(f"   cycles {sa['cycles']} / {sb['cycles']} rel {sa['rel_residual']:.3e} / "
              f"{sb['rel_residual']:.3e} free {free0} -> {free1}", flush=True)
        assert sa["cycles"] == sb["cycles"] and sa["rel_residual"] == sb["rel_residual"]
        assert np.array_equal(xa, xb)
        assert sb["rel_residual"] <= 1e-8
        if i > 0:  # (the first call may load the library's code for its kernels)
            assert free1 == free0  # the call allocated no device memory
    # the scratch keeps the last call's contents: a forced-cycle solve after
    # the others gives the same answer as the allocating call
    sa, sb, xa, xb, free0, free1 = _solve_both(nf, small, 4, forced=3)
    assert sa["cycles"] == sb["cycles"] == 3 and np.array_equal(xa, xb)
    assert free1 == free0


def test_noalloc_rejects_null_arguments(nf):
    g = nf.Grid(C.channel3d(64, 16, 16, Lx=1.28, Ly=0.32, Lz=0.32, n_levels=3))
    with pytest.raises(nf.NfvmError) as e:
        nf.nfvm_mg_solve_device_noalloc(g.h, 0, 0)
    assert e.value.status == nf.NFVM_E_INVAL
    g.close()
