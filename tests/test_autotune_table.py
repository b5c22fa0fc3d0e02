"""The tuned tile table as make_config reads it (CPU only): the nearest tuned edge per axis,
the batch shapes when asked for, the library defaults when the table lacks an entry, and an
explicit shape always winning.  The shapes change launches, never what is computed (the GPU
tests pin that); this checks only that the right shapes reach the configuration."""
import json

from paper_1410_4194_amd import autotune


def _table(tmp_path):
    t = {"fp64": {"32": {"y": 4, "z": 6, "x_rows": 2, "x_chunks": 1},
                  "256": {"y": 12, "z": 16, "x_rows": 1, "x_chunks": 8}},
         "fp32": {"64": {"y": 8, "z": 8}},
         "batch": {"fp64": {"march_seg": 12, "x_rows": 0, "x_chunks": 8}}}
    p = tmp_path / "tiles.json"
    p.write_text(json.dumps(t))
    return str(p)


def test_lookups_take_the_nearest_tuned_edge(tmp_path):
    path = _table(tmp_path)
    assert autotune.lookup(0, 40, 200, path) == (4, 16)     # y from edge 32, z from 256
    assert autotune.lookup_x(0, 300, 30, path) == (1, 8)    # by nx: nearest is 256
    assert autotune.lookup_x(0, 20, 20, path) == (2, 1)
    assert autotune.lookup_x(1, 64, 64, path) == (0, 0)     # no x entries: library choice
    assert autotune.lookup_batch(0, path) == (12, 0, 8)
    assert autotune.lookup_batch(1, path) is None
    assert autotune.lookup(0, 32, 32, str(tmp_path / "missing.json")) == (0, 0)


def test_make_config_uses_the_table_and_explicit_shapes_win(monkeypatch, tmp_path):
    path = _table(tmp_path)
    monkeypatch.setattr(autotune, "TABLE_PATH", path)
    for f in (autotune.lookup, autotune.lookup_x, autotune.lookup_batch):
        monkeypatch.setattr(f, "__defaults__", (path,))
    from paper_1410_4194_amd import ctu
    c = ctu.make_config(256, 256, 256, 1, 1, 1, 5 / 3)
    assert tuple(c.march_seg) == (12, 16) and (c.x_rows, c.x_chunks) == (1, 8)
    b = ctu.make_config(32, 32, 32, 1, 1, 1, 5 / 3, batch=True)
    assert tuple(b.march_seg) == (12, 12) and (b.x_rows, b.x_chunks) == (0, 8)
    e = ctu.make_config(32, 32, 32, 1, 1, 1, 5 / 3, march_seg=(7, 9), x_rows=3, x_chunks=2,
                        batch=True)
    assert tuple(e.march_seg) == (7, 9) and (e.x_rows, e.x_chunks) == (3, 2)
