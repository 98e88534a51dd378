"""Host-side logic: the open-channel timing workload has the paper's mesh
counts (Sec. 3.3, Table 1) and the boundary data of its verification case
(Sec. 3.1); the benchmark refuses more than one GPU."""
import numpy as np

from paper_2603_21869_amd import cases as C


def test_open_channel_mesh_counts_match_table1():
    # Table 1 lists 2,097,152, 8,388,608 and 33,554,432 cells for channel
    # lengths 0.64, 2.56 and 10.24 m on the 5 mm mesh (built without fields)
    for nx, L, cells in ((128, 0.64, 2097152), (512, 2.56, 8388608), (2048, 10.24, 33554432)):
        assert C.OPEN_CHANNEL_LENGTHS[nx] == L
        assert nx * 128 * 128 == cells
        assert abs(nx * 5e-3 - L) < 1e-12
    c = C.open_channel(128)
    assert c.ncells == 2097152 and c.h == (5e-3, 5e-3, 5e-3) and c.n_levels == 8
    assert c.n_steps == 100 and c.dt == 2e-3


def test_open_channel_boundaries():
    c = C.open_channel(32, 16, 16, h=0.04)
    kinds = {p.face: p for p in c.patches}
    assert kinds[0].kind == C.INLET and kinds[0].U == (0.1, 0.0, 0.0)
    assert abs(kinds[0].T - 298.15) < 1e-12
    assert kinds[1].kind == C.OUTLET
    for f in (2, 3, 4, 5):
        assert kinds[f].kind == C.WALL and abs(kinds[f].T_wall - 308.15) < 1e-12
    # Re = U L / nu with the 0.64 m cross-section gives the paper's 4384
    assert abs(0.1 * 0.64 / c.nu - 4384) < 1
    u = c.fields["u"]
    assert np.all(np.abs(u / 0.1 - 1) <= 0.01 + 1e-15) and u.std() > 0


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits with a message
    before any GPU work."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_bench_all_core_oracle_leg_runs_one_copy_per_core():
    """The all-core CPU leg starts one copy of the serial oracle per core
    (here two), each on the same sample, and reports their aggregate rate
    against the slowest copy; the workers never touch the GPU."""
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    from oracle import oracle as O
    O.build()
    case, _ = bench._cpu_sample("channel2d", 1e-6)
    r = bench.cpu_all_cores("channel2d", 1e-6, case.ncells, max_procs=2)
    ncores = min(2, len(os.sched_getaffinity(0)))
    assert r["cores"] == ncores and r["kind"] == "oracle" and r["unit"] == "Mcell-steps/s"
    assert r["value"] > 0 and f"{ncores} copies" in r["sample"]
