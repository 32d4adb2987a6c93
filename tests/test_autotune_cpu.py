"""Host logic of the launch-shape autotuner (no GPU)."""
from paper_2312_10318_amd import autotune


def test_candidates_cover_both_column_modes_on_even_widths():
    for has_mask in (False, True):
        shapes = autotune.candidates(4096, 4096, has_mask, "f32")
        one = [s for s in shapes if s[5] == 1]
        assert {s[3] for s in one} == {1, 2}
        assert {s[1] for s in one if s[3] == 1} == {1, 2, 4}
        assert {s[1] for s in one if s[3] == 2} == {1, 2, 4, 8, 16}
        assert {s[2] for s in shapes} == {0, 1}
        assert len(shapes) == len(set(shapes))
        assert all(len(s) == 7 and s[4] == 0 for s in shapes)
        assert all(s[6] == 0 for s in one)             # prefetch: two-step shapes only


def test_candidates_offer_two_steps_per_launch_where_it_applies():
    """FP32 and FP16 without a mask, any width: two-step shapes (at most four
    wavefronts per workgroup); masked and FP64 lattices: none."""
    for args in ((4096, 4096, False, "f32"), (4095, 4096, False, "f32"),
                 (4096, 4096, False, "f16")):
        two = [s for s in autotune.candidates(*args) if s[5] == 2]
        assert {s[0] for s in two} >= set(autotune.TB2_ROWS), args
        assert {s[1] for s in two} == {1, 2, 4}
        assert {s[6] for s in two} == {1, 2}           # loads one or two rows ahead
    for args in ((4096, 4096, True, "f32"), (4096, 4096, True, "f16"),
                 (4096, 4096, False, "f64")):
        assert all(s[5] == 1 for s in autotune.candidates(*args)), args


def test_candidates_offer_three_steps_per_launch_for_fp32():
    three = [s for s in autotune.candidates(4096, 4096, False, "f32") if s[5] == 3]
    assert {s[0] for s in three} == set(autotune.TB3_ROWS) | {25, 37, 74} | \
        set(autotune.whole_round_rows(4096, 4096, 116, 2, 2)) | \
        set(autotune.whole_round_rows(4096, 4096, 116, 1, 2))
    assert {s[1] for s in three} == {1, 2, 4} and {s[6] for s in three} == {1}
    for args in ((4096, 4096, False, "f16"), (4096, 4096, True, "f32"),
                 (4096, 4096, False, "f64")):
        assert all(s[5] != 3 for s in autotune.candidates(*args)), args


def test_candidates_respect_width_and_storage_limits():
    single = autotune.candidates(1025, 512, False, "f32")   # last strip: one column
    assert {s[3] for s in single if s[5] == 1} == {1}
    odd = autotune.candidates(1027, 512, True, "f32")
    assert {s[3] for s in odd} == {1, 2}
    f64 = autotune.candidates(4096, 4096, False, "f64")
    assert max(s[1] for s in f64 if s[3] == 2) == 8
    short = autotune.candidates(256, 8, False, "f16")
    assert max(s[0] for s in short) == 8
    assert max(s[0] for s in autotune.candidates(256, 8, False, "f32") if s[5] == 2) == 8


def test_cache_key_buckets_sizes():
    assert autotune.key(4000, 4100, "f32", False) == autotune.key(4096, 4096, "f32", False)
    assert autotune.key(4096, 4096, "f32", True) != autotune.key(4096, 4096, "f32", False)
    keys = {autotune.key(4096, 4096, "f32", m, walls=w) for m, w in
            ((False, False), (True, False), (True, True))}
    assert len(keys) == 3


def test_whole_row_walls_get_multi_step_candidates():
    """A mask whose solid nodes fill whole rows: FP32 and FP16 lattices are
    offered the multi-step shapes of open lattices; FP64 keeps one step."""
    import numpy as np
    for storage in ("f32", "f16", "f64"):
        walls = autotune.candidates(4096, 4096, True, storage, walls=True)
        open_ = autotune.candidates(4096, 4096, False, storage)
        assert sorted(walls) == sorted(open_)
    assert all(s[5] == 1 for s in autotune.candidates(4096, 4096, True, "f16"))
    m = np.zeros((10, 7), np.uint8)
    assert autotune.row_walls(m)
    m[[0, 9]] = 1
    assert autotune.row_walls(m) and not autotune.row_walls(m, inflow=(0.01, 1.0, 1.0))
    m[4, 3] = 1
    assert not autotune.row_walls(m)
    m = np.zeros((10, 7), np.uint8)
    m[:, 0] = 1                       # a wall along y
    assert not autotune.row_walls(m) and not autotune.row_walls(None)


def test_build_reads_register_spills_from_compiler_remarks():
    from paper_2312_10318_amd import build
    text = "\n".join([
        "a.hip:1:1: remark: Function Name: _Z5sweepv [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs: 207 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     SGPRs Spill: 7 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs Spill: 56 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: _Z4initv [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert build.spills(text) == {"_Z5sweepv": 56, "_Z4initv": 0}


def test_batch_candidates_and_key():
    shapes = autotune.batch_candidates()
    assert (0, 4, 0, 0, -1, 1) in shapes                # the library's batch default
    assert {s[1] for s in shapes} <= {1, 2, 4}           # batched workgroups hold at most 4
    assert {s[3] for s in shapes} == {0}                 # members keep their column mode
    # row policies: each member's own rows, or a batch-wide cap; both orders
    assert {s[4] for s in shapes if s[0] == 0} == {-1, 16384, 32768}
    assert {s[5] for s in shapes} == {1, 2}
    assert len(shapes) == len(set(shapes))
    a = autotune.batch_key([(64, 64), (1000, 1000), (1024, 1024)], "f32", False)
    b = autotune.batch_key([(1024, 1024), (64, 64), (1010, 1000)], "f32", False)
    assert a == b                                        # order and small size changes
    assert a != autotune.batch_key([(64, 64), (1000, 1000)], "f32", False)
    assert a != autotune.batch_key([(64, 64), (1000, 1000), (1024, 1024)], "f16", False)
    assert a != autotune.batch_key([(64, 64), (1000, 1000), (1024, 1024)], "f32", True)


def test_cache_round_trip_and_unwritable_location(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.save_cache({"k": {"best": [1, 2]}}, path)
    assert autotune.load_cache(path) == {"k": {"best": [1, 2]}}
    blocker = tmp_path / "file"
    blocker.write_text("x")
    # a directory that cannot be created (a file is in the way): no exception
    assert autotune.save_cache({"k": 1}, str(blocker / "tune.json")) is False
    assert autotune.load_cache(str(blocker / "tune.json")) == {}


def test_whole_round_rows():
    """Rows that make the workgroups fill the resident slots in whole rounds:
    4096^2, three steps per launch (36 windows of 116 columns, 9 groups of
    four wavefronts, 512 resident workgroups): 56, 113 and 170 row blocks."""
    assert autotune.whole_round_rows(4096, 4096, 116, 4, 2) == [25, 37, 74]
    for k, r in zip((3, 2, 1), (25, 37, 74)):
        blocks = -(-4096 // r)
        assert blocks * 9 <= k * 512 < (-(-4096 // (r - 1))) * 9 or r == 8
    assert autotune.whole_round_rows(64, 8, 116, 4, 2) == []   # rows above the height
