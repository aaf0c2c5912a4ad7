"""Ray launching (Sec. III-A): icosahedron with 20 faces and 12 vertices,
faces subdivided, rays through the vertices."""
import numpy as np
import pytest

from rtgen import icosphere as ico


@pytest.mark.parametrize("level", [0, 1, 2, 3, 5])
def test_counts_and_euler(level):
    v = ico.directions(level)
    f = ico.faces(level)
    assert v.shape == (10 * 4 ** level + 2, 3)
    assert f.shape == (20 * 4 ** level, 3)
    edges = {tuple(sorted(e)) for tri in f for e in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0]))}
    assert v.shape[0] - len(edges) + f.shape[0] == 2      # Euler characteristic of a sphere


def test_config_counts():
    assert ico.vertex_count(5) == 10_242
    assert ico.vertex_count(9) == 2_621_442


@pytest.mark.parametrize("level", [0, 3, 6])
def test_unit_norm_and_float32(level):
    v = ico.directions(level)
    n = np.sqrt((v * v).sum(1))
    assert np.max(np.abs(n - 1.0)) < 4e-16
    v32 = v.astype(np.float32).astype(np.float64)
    n32 = np.sqrt((v32 * v32).sum(1))
    assert np.max(np.abs(n32 - 1.0)) < 2 ** -23


@pytest.mark.parametrize("level", [0, 2, 4])
def test_central_symmetry(level):
    v = ico.directions(level)
    key = {tuple(np.round(p, 12)) for p in v}
    assert all(tuple(np.round(-p, 12)) in key for p in v)


def test_prefix_property():
    big = ico.directions(6)
    for lv in range(6):
        small = ico.directions(lv)
        assert np.array_equal(big[: small.shape[0]], small)


@pytest.mark.parametrize("level", [1, 3])
def test_valence(level):
    f = ico.faces(level)
    nv = ico.vertex_count(level)
    val = np.bincount(f.ravel(), minlength=nv)
    assert np.sum(val == 5) == 12 and np.sum(val == 6) == nv - 12


def test_level0_is_regular_icosahedron():
    v = ico.directions(0)
    d = np.sqrt(((v[:, None] - v[None]) ** 2).sum(-1))
    edge = d[d > 1e-9].min()
    assert np.sum(np.abs(d - edge) < 1e-12) == 60           # 30 edges, counted twice
    assert np.allclose(edge, 1.0514622242382672)            # 4 / sqrt(10 + 2 sqrt 5)


def test_spacing_and_rays():
    assert abs(np.degrees(ico.angular_spacing(0)) - 63.43494882) < 1e-6
    r = ico.make_rays((1, 2, 3), ico.directions(1), 1e-4, 50.0)
    assert r.dtype == np.float32 and r.shape == (42, 8)
    assert np.all(r[:, 0:3] == np.float32([1, 2, 3])) and np.all(r[:, 3] == np.float32(1e-4))
    first = ico.directions_n(100)
    assert first.shape == (100, 3) and np.array_equal(first, ico.directions(3)[:100])


@pytest.mark.parametrize("level", [0, 2, 4])
def test_edge_angles(level):
    a = ico.edge_angles(level)
    assert a.size == 30 * 4 ** level                        # E = 3F / 2
    # level 0: every edge subtends arccos(1/sqrt(5)); later levels split each
    # edge in two, so angles shrink by about half per level
    assert abs(a.min() - ico.angular_spacing(level)) < 1e-12
    assert a.max() < 1.25 * ico.angular_spacing(level)
