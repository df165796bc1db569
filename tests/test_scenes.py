"""The seeded input generators: determinism, sizes and validity of every config."""
import numpy as np
import pytest

import oracle
import scenes


@pytest.fixture(scope="module")
def medium():
    return scenes.medium()


def test_tiny_is_deterministic_and_sized():
    a, b = scenes.tiny(), scenes.tiny()
    assert scenes.digest(a) == scenes.digest(b)
    assert scenes.digest(scenes.tiny(seed=9)) != scenes.digest(a)
    assert a["rest"].shape == (250, 3) and a["tets"].shape == (768, 4)
    assert len(a["pt"]) == 25 and len(a["ee"]) == 40 and a["fixed"].sum() == 25
    assert a["kappa"] == 1e4 and a["delta"] == 1e-3 and a["dt"] == 0.01


def test_medium_sizes(medium):
    assert medium["rest"].shape == (26620, 3) and medium["tets"].shape == (120000, 4)
    assert len(medium["pt"]) == 12000 and len(medium["ee"]) == 8000
    assert medium["fixed"].sum() == 0
    E = np.unique(medium["E"])
    assert len(E) == 20 and E.min() >= 1e4 and E.max() <= 1e6


@pytest.mark.parametrize("which", ["tiny", "shifted", "medium", "serve"])
def test_states_and_constraints_are_valid(which, medium):
    sc = {"tiny": scenes.tiny, "shifted": lambda: scenes.tiny(lateral=(0.37, 0.21)),
          "medium": lambda: medium, "serve": lambda: scenes.serve_request(3)}[which]()
    st = oracle.prepare(sc)
    for x in (sc["x"], sc["x_hat"]):
        F = oracle.deformation_gradient(x, st.tets, st.Dminv)
        assert np.linalg.det(F).min() > 0
    C = np.concatenate([sc["pt"], sc["ee"]])
    assert all(len(set(r)) == 4 for r in C.tolist())
    ids, d, n, w = oracle.linearize(sc["x"], sc["pt"], sc["ee"])
    assert d.min() > 0
    assert np.all(sc["x_hat"][sc["fixed"].astype(bool)] == sc["x"][sc["fixed"].astype(bool)])


def test_shifted_tiny_covers_interior_point_triangle_cases():
    sc = scenes.tiny(lateral=(0.37, 0.21))
    ids, d, n, w = oracle.linearize(sc["x"], sc["pt"], sc["ee"])
    npt = len(sc["pt"])
    interior = np.all(np.abs(w[:npt, 1:]) > 1e-9, axis=1)
    interior_ee = np.all(np.abs(w[npt:]) > 1e-9, axis=1)
    assert interior.any() and interior_ee.any()


def test_serve_request_sizes():
    for i in range(6):
        sc = scenes.serve_request(i)
        n_c = len(sc["pt"]) + len(sc["ee"])
        assert 174 <= n_c <= 4038
        assert 2592 <= len(sc["tets"]) <= 12 * 29 ** 3
