"""Finite-difference pins of the FP64 NumPy reference of the warm-start network (no GPU)."""

import numpy as np

from oracle import cnn as ref


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(1, 2, 4, 5))
    w = rng.normal(size=(3, 2, 3, 3))
    b = rng.normal(size=3)
    y = ref.conv3x3(x, w, b)
    o, i, j = 2, 0, 4  # a corner pixel (zero padding enters)
    s = b[o]
    for c in range(2):
        for u in range(3):
            for v in range(3):
                ii, jj = i + u - 1, j + v - 1
                if 0 <= ii < 4 and 0 <= jj < 5:
                    s += w[o, c, u, v] * x[0, c, ii, jj]
    assert abs(y[0, o, i, j] - s) < 1e-13


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    layers = [(rng.normal(size=(4, 3, 3, 3)) * 0.5, rng.normal(size=4) * 0.1, True),
              (rng.normal(size=(2, 4, 3, 3)) * 0.5, rng.normal(size=2) * 0.1, False)]
    x = rng.normal(size=(2, 3, 6, 7))
    t = rng.normal(size=(2, 2, 6, 7))
    fl = (rng.random((2, 6, 7)) < 0.7).astype(float)

    def loss_of(L):
        return ref.masked_mse(ref.forward(L, x)[-1], t, fl)[0]

    acts = ref.forward(layers, x)
    _, g = ref.masked_mse(acts[-1], t, fl)
    grads = ref.backward(layers, x, acts, g)
    h = 1e-6
    for li in range(2):
        for idx in [(0, 0, 0, 0), (1, 2, 1, 2), (1, 1, 2, 0)]:
            if idx[0] >= layers[li][0].shape[0] or idx[1] >= layers[li][0].shape[1]:
                continue
            Lp = [(w.copy(), b.copy(), r) for w, b, r in layers]
            Lm = [(w.copy(), b.copy(), r) for w, b, r in layers]
            Lp[li][0][idx] += h
            Lm[li][0][idx] -= h
            fd = (loss_of(Lp) - loss_of(Lm)) / (2 * h)
            assert abs(fd - grads[li][0][idx]) < 1e-6 * max(1.0, abs(fd))
        Lp = [(w.copy(), b.copy(), r) for w, b, r in layers]
        Lm = [(w.copy(), b.copy(), r) for w, b, r in layers]
        Lp[li][1][0] += h
        Lm[li][1][0] -= h
        fd = (loss_of(Lp) - loss_of(Lm)) / (2 * h)
        assert abs(fd - grads[li][1][0]) < 1e-6 * max(1.0, abs(fd))


def test_feature_profiles_reduce_to_special_cases():
    """No solid: the porosity-weighted profile is the profile itself; every column half solid:
    its increments double."""
    rng = np.random.default_rng(3)
    W, H = 12, 8
    X_in = np.array([[0.5, 0.3, 0.2]])
    prof = X_in[:, :2, None] - np.cumsum(rng.uniform(0, 1e-3, (1, 2, W)), axis=2)
    prof[:, :, 0] = X_in[:, :2]
    f, base = ref.features(np.zeros((1, H, W), np.uint8), X_in, np.array([1.0]), prof)
    assert np.allclose(base, prof, atol=1e-15) and np.all(f[0, 7] == 1.0)
    solid = np.zeros((1, H, W), np.uint8)
    solid[:, ::2, :] = 1
    f, base = ref.features(solid, X_in, np.array([1.0]), prof)
    assert np.allclose(base - X_in[:, :2, None], 2.0 * (prof - X_in[:, :2, None]), atol=1e-15)
    assert np.allclose(f[0, 5:7], ((base[0] - X_in[0, :2, None]) / 0.01)[:, None, :], atol=1e-12)
    assert np.array_equal(f[0, 0], 1.0 - solid[0]) and np.all(f[0, 3] == 0.5)
    assert np.all(f[0, 1] == 0.5) and np.all(f[0, 2] == 0.3) and np.all(f[0, 7] == 0.5)
    assert f[0, 4, 0, 0] == 0.0 and f[0, 4, 0, -1] == 1.0


def test_assemble_stays_on_the_simplex():
    rng = np.random.default_rng(4)
    pred = rng.normal(0.0, 5.0, (2, 2, 4, 6))
    prof = np.full((2, 2, 6), 0.4)
    X = ref.assemble(pred, prof, 0.1, 1e-6)
    assert np.all(X >= 1e-6 - 1e-15) and np.allclose(X.sum(axis=1), 1.0, atol=1e-15)
