"""Host logic of the autotuner's shapes (no GPU): names round-trip, and every
candidate is one the library accepts (tile sides 8, 16 or 32; a blend split
of 1, 2 or 4 that divides the tile height into parts of at least 8 rows)."""
import os
import sys

from paper_2501_17792_amd import autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_shape_names_round_trip():
    for tw, th, split in autotune.CANDIDATES:
        name = autotune.shape_name(tw, th, split)
        assert autotune.parse_shape(name) == ((tw, th), split)
    assert autotune.shape_name(16, 32) == "16x32" and autotune.parse_shape("16x32") == ((16, 32), 1)
    assert autotune.parse_shape("32x32s4") == ((32, 32), 4)


def test_candidates_are_valid_library_options():
    assert len(set(autotune.CANDIDATES)) == len(autotune.CANDIDATES)
    for tw, th, split in autotune.CANDIDATES:
        assert tw in (8, 16, 32) and th in (8, 16, 32)
        assert split in (1, 2, 4) and th % split == 0 and th // split >= 8


def test_counter_measurements_name_candidate_shapes():
    sys.path.insert(0, ROOT)
    import bench

    for key in bench.MEASURED["tiles"]:
        assert key in autotune.CANDIDATES


def test_frame_roofline_uses_counters_of_the_timed_shape_only():
    """The bench's roofline object takes counter traffic and VALU issue only
    for the tile shape and split they were measured at (and these sources):
    compositing dominant here, its FP32 work against 78.6 TFLOP/s."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2501_17792_amd import synth

    scene = synth.scene_c1()
    stats = dict(n_splats=1_000_000, n_pairs=2_000_000)
    stage = {"project_fused": 0.5, "segsort": 0.4, "blend": 1.0}
    blend = {"evals_per_frame": 10_000_000}
    measured = next(iter(bench.MEASURED["tiles"]))
    ok = bench.kernel_digest() == bench.MEASURED["digest"]
    r = bench.frame_roofline(stage, stats, scene, 0, measured[:2], measured[2], blend)
    assert r["bound"] == "alu" and r["kernel"] == "blend_kernel"
    assert abs(r["achieved"] - 10_000_000 * bench.BLEND_FLOPS_PER_EVAL / 1e-3 / 1e12) < 1e-3
    assert (r["traffic"] is not None) == ok and ("issue" in r) == ok
    other = (16, 16, 1) if measured != (16, 16, 1) else (32, 16, 1)
    r2 = bench.frame_roofline(stage, stats, scene, 0, other[:2], other[2], blend)
    assert r2["traffic"] is None and "issue" not in r2
