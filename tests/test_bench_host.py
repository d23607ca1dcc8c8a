"""CPU checks of the benchmark's host logic: the profile lookup that supplies measured HBM
traffic keys on the kernel code with its comments removed."""
import bench


def test_comments_do_not_change_the_kernel_hash():
    a = "int f(int x) {  // one\n  return x + 1; /* two\n lines */\n}\n"
    b = "// header\nint f(int x) {\n  return x + 1;\n}\n"
    assert bench.code_without_comments(a) == bench.code_without_comments(b)
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench.code_without_comments(a) != bench.code_without_comments(c)


def test_profile_lookup_matches_tuning_exactly():
    t = {k: dict(bench.BENCH_TUNING, pack_skew=0, wave_width=0)[k] for k in bench.TUNING_KEYS}
    found = bench.profiled_counters("k_step_packs", t)
    other = bench.profiled_counters("k_step_packs", dict(t, lds_width=t["lds_width"] - 16))
    assert other is None
    assert found is None or found["hbm_bytes_per_launch"] > 0


def test_workload_shape_statistics_on_known_trees():
    # a 5-segment chain (depth 5, one tip) and a tree of a root with three children, the
    # middle one with two children of its own (depth 3, widest level 3, four tips)
    import dataclasses

    import numpy as np

    from orchard_inputs import assemble, chain_tree
    a = chain_tree(5, length=0.1, radius=0.02)
    b = dataclasses.replace(chain_tree(6, length=0.1, radius=0.01),
                            parent=np.array([-1, 0, 0, 0, 2, 2], np.int32))
    s = bench.workload_stats(assemble([a, b]))
    assert (s["max_depth"], s["mean_depth"], s["widest_level"], s["tips"]) == (5, 4.0, 3, 5)
    assert abs(s["r_tip_mm"] - (20.0 + 4 * 10.0) / 5) < 1e-9


def test_sphere_fit_profile_record_keys_on_its_source():
    # the sphere-fit summary's counters apply only while its kernel source (comments aside)
    # is the profiled one
    rec = bench.profiled_counters("k_sphere_fit", None, bench.SPHERE_SOURCES)
    assert rec is None or (rec["valu_insts_per_launch"] > 0 and rec["hbm_bytes_per_launch"] > 0)
    assert bench.profiled_counters("k_sphere_fit", None, bench.STEP_SOURCES) is None
