"""Host-side helpers that need no GPU: the bench's mesh adjacency, its
paper-context ratios and traffic bookkeeping, and the synthetic
reconstruction inputs."""
import numpy as np

from graphs import grid_graph
from paper_2511_22094_amd import synth


def test_bench_grid_csr_is_the_six_neighbourhood_graph():
    import bench
    shape = (3, 4, 5)
    rp, col = bench.grid_csr(shape)
    r2, c2 = grid_graph(np.ones(shape, np.uint8), 3)
    assert np.array_equal(rp, r2)
    for i in range(rp.size - 1):
        assert sorted(col[rp[i]:rp[i + 1]]) == sorted(c2[r2[i]:r2[i + 1]])
    # symmetric, no self loops
    pairs = {(i, int(j)) for i in range(rp.size - 1) for j in col[rp[i]:rp[i + 1]]}
    assert all((j, i) in pairs for i, j in pairs) and all(i != j for i, j in pairs)


def test_caipi_mask_pattern():
    """R_y = 1, R_z = 9, z-shift 3 per line, TE-shift 2 per echo."""
    m = synth.caipi_mask(6, 27, 36)
    assert m.dtype == np.uint8 and m.shape == (6, 27, 36)
    # every line samples every ninth z position
    assert np.all(m.sum(axis=2) == 36 // 9)
    for e in range(6):
        for y in range(27):
            z = np.flatnonzero(m[e, y])
            assert np.all(np.diff(z) == 9) and (z[0] - 3 * y - 2 * e) % 9 == 0
    assert m.mean() == 1 / 9


def test_sense_draw_is_seeded_and_shaped():
    a = synth.sense_draw(3, 2, 4, 16, 32)
    b = synth.sense_draw(3, 2, 4, 16, 32)
    assert a.truth.shape == (2, 16, 32) and a.coils.shape == (4, 16, 32)
    assert a.noise.shape == (2, 4, 16, 32) and a.mask.shape == (2, 16, 32)
    assert np.array_equal(a.truth, b.truth) and np.array_equal(a.noise, b.noise)
    assert np.abs(a.coils).max() <= 1.0 + 1e-12


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU; asking for more exits with a message and
    status 2 before touching a device."""
    import subprocess
    import sys
    from pathlib import Path
    root = Path(__file__).resolve().parents[1]
    r = subprocess.run([sys.executable, str(root / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_paper_context_ratios():
    """The speed-ups over one oracle core are this build's GPU rates over the
    single-thread oracle rates, set beside the paper's quoted figures."""
    import bench
    mh = {"value": 6.0e10}
    cpu = {"value": 1.6e7, "single_thread": {"value": 1.0e6}}
    adam = {"value": 9.0e9}
    adam_err = {"cpu_oracle": {"single_thread": {"value": 6.0e5}}}
    c = bench.paper_context(mh, cpu, adam, adam_err)
    assert c["mh_gre3_vs_one_oracle_core"] == 6.0e4
    assert c["adam_tv_dwi2_vs_one_oracle_core"] == 1.5e4
    assert c["paper_mh_nexi_vs_one_cpu_core"] == 14380
    assert c["paper_adam_nexi_vs_one_cpu_core"] == 451
    # without the CPU baseline there is no ratio to give
    assert bench.paper_context(mh, None, adam, adam_err) is None
    assert "adam_tv_dwi2_vs_one_oracle_core" not in bench.paper_context(mh, cpu, None, None)


def test_bench_measured_traffic_follows_the_kernel_sources(monkeypatch):
    """Counter-based traffic is reported only for the sources it was taken
    on: a different recorded hash gives null."""
    import copy
    import bench
    table = copy.deepcopy(bench.MEASURED_TRAFFIC)
    key = "fit_step"
    table[key]["sha256"] = "0" * 64
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", table)
    assert bench.measured_traffic(key) is None
    assert bench.measured_traffic("no such kernel") is None
