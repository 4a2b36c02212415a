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
