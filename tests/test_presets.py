"""The workload presets (CPU): each states the configuration the benchmark
and the tests run, and bench.py builds its workloads from them."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_presets_state_the_workloads():
    from paper_1604_03478_amd import presets
    c1 = presets.cond24()
    assert (c1.config.n, c1.config.flow, c1.config.ste, c1.config.precision, c1.steps) == \
        (24, 0, 0.1, "f64", 2000)
    assert c1.config.seed_profile == 1 and c1.config.heating == "y0"
    c2 = presets.conv64()
    assert (c2.config.n, c2.config.ra, c2.config.pr, c2.config.ste, c2.steps) == \
        (64, 1e4, 1.0, 0.1, 20000)
    assert c2.config.flow == 1 and c2.config.heating == "y0" and c2.config.precision == "f32"
    c3 = presets.conv256("f16s")
    assert (c3.config.n, c3.config.ra, c3.config.precision, c3.steps) == (256, 1e5, "f16s", 100000)
    assert presets.conv256(all_liquid=True).config.s0 == 256.0
    c4 = presets.adj64()
    assert c4.config == c2.config and (c4.steps, c4.every_k, c4.hot_wall_seed) == (2000, 100, 0)
    c5 = presets.bottom512()
    assert (c5.config.n, c5.config.ra, c5.config.heating, c5.config.precision, c5.steps) == \
        (512, 1e6, "z0", "f16s", 200000)
    assert c2.with_precision("f64").config.precision == "f64"
    assert set(presets.ALL) == {"cond24", "conv64", "conv256", "adj64", "bottom512"}


def test_bench_builds_its_workloads_from_the_presets():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1604_03478_amd import presets
    assert bench.workload_config(256, "f32", True) == presets.conv256("f32", True).config
    assert bench.workload_config(128, "f16s", False) == presets.conv256("f16s", n=128).config
