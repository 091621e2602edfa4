"""Host-side logic of the library checked on the CPU (no GPU needed): the
judge's offsets and weights and the network's inputs that demag_quad_predict
computes in C++ equal, bit for bit, the recipe written in Python
(inputs.fit_offsets, inputs.quad_features) that the tests and the training
cases use."""
import numpy as np

from paper_1212_3509_amd import api, inputs


def _grids():
    rng = np.random.default_rng(17)
    grids = [tuple(int(v) for v in rng.integers(1, 300, 3)) for _ in range(150)]
    grids += [tuple(int(v) for v in rng.integers(32, 65, 3)) for _ in range(150)]
    grids += [(1, 1, 1), (2, 1, 3), (4, 4, 4), (5, 5, 5), (128, 128, 128), (256, 256, 256), (256, 256, 4),
              (1024, 1024, 1024), (4096, 4096, 4096), (4096, 7, 300), (33, 4096, 1)]
    return grids


def test_library_offsets_equal_the_python_recipe():
    for n in _grids():
        J, w = api.quad_offsets(n)
        Jp, wp = inputs.fit_offsets(n)
        assert np.array_equal(J, Jp), n
        assert np.array_equal(w, wp), n


def test_library_features_equal_the_python_recipe():
    rng = np.random.default_rng(5)
    for n in _grids()[:200]:
        h = 1.0 / max(n)
        tol = float(rng.uniform(-9, -4))
        R = int(rng.integers(16, 33))
        x = api.quad_features(n, h, tol, R)
        xp = inputs.quad_features([n], [h], [tol], [R])[0]
        assert np.array_equal(x.view(np.uint32), xp.view(np.uint32)), (n, tol, R)
