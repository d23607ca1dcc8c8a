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
