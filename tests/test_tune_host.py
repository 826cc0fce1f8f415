"""CPU checks of the launch table (abcs_set_launch_table and friends, host
code only) and of the tuner's host logic."""
import json

import numpy as np
import pytest


@pytest.fixture()
def g():
    import paper_2001_09632_amd as g
    g.set_launch_table([])
    yield g
    g.set_launch_table([])


def test_table_set_read_reset(g):
    g.set_launch_table([dict(block=16, transform="dct", precision="bf16x3", size_class=1, split=2),
                        dict(block=8, transform="wht", precision="fp32", size_class=3, split=1)])
    assert g.launch_split(16, "dct", "bf16x3", 1) == 2
    assert g.launch_split(16, "dct", "fp32", 1) == 0
    assert g.launch_split(8, "wht", "fp32", 3) == 1
    # Walsh-Hadamard launches run in float32 and read the float32 entry
    assert g.launch_split(8, "wht", "bf16", 3) == 1
    # a new table replaces the old one
    g.set_launch_table([dict(block=32, transform="dct", precision="fp16", size_class=0, split=1)])
    assert g.launch_split(16, "dct", "bf16x3", 1) == 0
    assert g.launch_split(32, "dct", "fp16", 0) == 1
    g.set_launch_table([])
    assert g.launch_split(32, "dct", "fp16", 0) == 0


@pytest.mark.parametrize("bad", [dict(block=12), dict(split=3), dict(split=-1), dict(size_class=4),
                                 dict(precision=7), dict(transform=2)])
def test_table_rejects_bad_entries_and_keeps_the_old_one(g, bad):
    g.set_launch_table([dict(block=16, transform="dct", precision="fp32", size_class=2, split=1)])
    e = dict(block=16, transform="dct", precision="fp32", size_class=0, split=1)
    e.update(bad)
    with pytest.raises(g.AbcsError, match="EINVAL"):
        g.set_launch_table([e])
    assert g.launch_split(16, "dct", "fp32", 2) == 1
    with pytest.raises(g.AbcsError, match="EINVAL"):
        g.launch_split(12, "dct", "fp32", 0)


def test_build_id_is_the_hash_of_the_sources():
    import paper_2001_09632_amd as g
    from paper_2001_09632_amd import build
    assert g.build_id() == build.build_id()


def test_code_text_drops_comments_only():
    from paper_2001_09632_amd.build import code_text
    src = (b'int a = 1; // one\n/* two\n   lines */ const char* s = "x // y /* z */";\n'
           b"char q = '\"'; char e = '\\''; /* c */ int b; \n\n  \n#define M(x) (x) // m\n")
    assert code_text(src) == (b'int a = 1;\n  const char* s = "x // y /* z */";\n'
                              b"char q = '\"'; char e = '\\'';   int b;\n#define M(x) (x)")
    # a changed token changes the text; a changed comment does not
    assert code_text(src.replace(b"int b", b"int c")) != code_text(src)
    assert code_text(src.replace(b"two", b"three")) == code_text(src)


def test_stored_table_of_another_build_is_ignored(g, tmp_path):
    from paper_2001_09632_amd import tune
    e = dict(block=16, transform="dct", precision="fp32", size_class=3, split=1, ms=[1.0, 0.5, 0.6])
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"build_id": "not-this-build", "entries": [e]}))
    assert tune.load(str(p)) is None
    assert g.launch_split(16, "dct", "fp32", 3) == 0
    p.write_text(json.dumps({"build_id": g.build_id(), "entries": [e]}))
    assert tune.load(str(p)) is not None
    assert g.launch_split(16, "dct", "fp32", 3) == 1


def test_tuning_batches_land_in_their_size_class():
    """Each tuning batch has the tile count of its size class (tiles of up to
    16 blocks along a block row)."""
    from paper_2001_09632_amd import tune
    bounds = (0, 256, 2048, 16384, 1 << 40)
    for B, batches in tune.BATCHES.items():
        for sc, (n, side) in enumerate(batches):
            tiles = n * (side // B) * -(-(side // B) // 16)
            assert bounds[sc] <= tiles < bounds[sc + 1], (B, sc, tiles)


def test_smooth_images_are_seeded():
    from paper_2001_09632_amd import tune
    a = tune.smooth_images(2, 64)
    b = tune.smooth_images(2, 64)
    assert a.dtype == np.uint8 and a.shape == (2, 64, 64) and np.array_equal(a, b)
    assert a.std() > 10


def test_binding_installs_the_stored_table_of_its_build(g, tmp_path, monkeypatch):
    """Loading the library installs tuned_launch.json when it belongs to
    this build, and ignores it otherwise."""
    from paper_2001_09632_amd import _native
    e = dict(block=32, transform="dct", precision="bf16", size_class=2, split=2, ms=[1.0, 0.9, 0.8])
    p = tmp_path / "tuned.json"
    monkeypatch.setattr(_native, "TUNED_PATH", str(p))
    p.write_text(json.dumps({"build_id": "another-build", "entries": [e]}))
    _native._install_tuned_launches(_native.lib())
    assert g.launch_split(32, "dct", "bf16", 2) == 0
    p.write_text(json.dumps({"build_id": g.build_id(), "entries": [e]}))
    _native._install_tuned_launches(_native.lib())
    assert g.launch_split(32, "dct", "bf16", 2) == 2
