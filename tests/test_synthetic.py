"""Input generators: shapes, seeding and the structure the paper fixes."""
import numpy as np

import synthetic as S


def test_links_are_su3_and_seeded():
    U = S.gauge_links((3, 4, 2, 5), 0.3, 7)
    assert U.shape == (4, 5, 2, 4, 3, 3, 3)
    eye = np.einsum("...ab,...cb->...ac", U, U.conj())
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    assert np.array_equal(U, S.gauge_links((3, 4, 2, 5), 0.3, 7))
    assert not np.array_equal(U, S.gauge_links((3, 4, 2, 5), 0.3, 8))


def test_point_sources_match_sec2():
    dims = (2, 3, 2, 2)
    B = S.point_sources(dims).reshape(S.volume(dims), 4, 3, 12)
    assert B.sum() == 12
    for s in range(4):
        for c in range(3):
            # s^(i)(origin, alpha, a) = 1 iff i = a + 3 (alpha - 1)  (1-based)
            assert B[0, s, c, c + 3 * s] == 1
    assert np.abs(B[1:]).sum() == 0


def test_noise_sources():
    z = S.z2_sources((2, 2, 2, 2), 5, 41)
    assert set(np.unique(z.real).tolist()) == {-1.0, 1.0} and np.all(z.imag == 0)
    g = S.gaussian_sources((2, 2, 2, 2), 5, 51)
    assert g.shape == (2, 2, 2, 2, 4, 3, 5)
    assert abs(np.std(g.real) - 1) < 0.2


def test_random_su3():
    O = S.random_su3((10,), 3)
    assert np.abs(np.linalg.det(O) - 1).max() < 1e-13
    assert np.abs(O @ np.conj(np.swapaxes(O, -1, -2)) - np.eye(3)).max() < 1e-13
