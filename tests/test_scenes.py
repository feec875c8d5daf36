"""The seeded input generators: deterministic, and at the stated sizes."""
import numpy as np

import rpr_scenes as R


def test_tiny_is_12_triangles():
    c = R.tiny_config()
    assert c["tris"].shape == (12, 3) and c["verts"].dtype == np.float32
    assert np.allclose(c["verts"].min(0), 0) and np.allclose(c["verts"].max(0), [10, 7, 3])


def test_city_size_and_determinism():
    a = R.city_config()
    b = R.city_config()
    assert np.array_equal(a["verts"], b["verts"]) and np.array_equal(a["tris"], b["tris"])
    assert abs(len(a["tris"]) - 100_000) < 2_000
    assert a["sources"].shape == (8, 3)
    assert a["absorption"].shape == (8, 4)
    assert (a["absorption"] >= 0.05).all() and (a["absorption"] <= 0.5).all()


def test_learn_room_ranges():
    for s in range(10000, 10020):
        r = R.learn_room(s)
        assert r["kind"] in ("shoebox", "lroom")
        assert (r["dims"] >= 3).all() and (r["dims"] <= 40).all()
        assert np.linalg.norm(r["sources"][0] - r["listener"]) >= 1.0
