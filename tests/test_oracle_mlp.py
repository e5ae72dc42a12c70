"""Pins of the float64 surrogate MLP: its hand-written backward pass against
central finite differences, and the tanh-form GELU against the erf form."""
import math

import numpy as np

from oracle import mlp


def _problem(seed=0, n=48):
    rng = np.random.default_rng(seed)
    theta = rng.normal(scale=0.05, size=mlp.param_count())
    Bf = rng.normal(scale=2.0, size=(mlp.N_FREQ, mlp.N_IN))
    v = rng.uniform(-1, 1, size=(n, 5))
    t = rng.normal(scale=3.0, size=n)
    m = (rng.random(n) < 0.8).astype(np.float64)
    return theta, Bf, v, t, m


def test_param_count_matches_layout():
    assert mlp.param_count() == 128 * 256 + 256 + 3 * (256 * 256 + 256) + 256 + 1 == 230_657


def test_backward_matches_central_differences():
    theta, Bf, v, t, m = _problem()
    y, cache = mlp.forward(theta, v, Bf)
    g = mlp.backward(theta, cache, y, t, m)
    rng = np.random.default_rng(1)
    # 10 random parameters plus one of every layer's bias and the head bias
    idx = list(rng.choice(theta.size, size=10, replace=False)) + [32768, 33024 + 65536, theta.size - 1]
    for i in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(mlp.forward(tp, v, Bf)[0], t, m) - mlp.loss(mlp.forward(tm, v, Bf)[0], t, m)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_gelu_tanh_form_close_to_erf_form_and_derivative():
    x = np.linspace(-6, 6, 2001)
    erf_form = 0.5 * x * (1 + np.vectorize(math.erf)(x / math.sqrt(2)))
    assert np.max(np.abs(mlp.gelu(x) - erf_form)) < 1e-3
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def test_features_are_unit_circle_pairs():
    theta, Bf, v, t, m = _problem()
    f = mlp.features(v, Bf)
    assert f.shape == (v.shape[0], 128)
    assert np.allclose(f[:, :64] ** 2 + f[:, 64:] ** 2, 1.0)


def test_free_space_prior_equals_image_method_line_of_sight():
    """The prior's definition against the oracle's image-method LoS path
    (isotropic antennas, no obstacle): 10 log10 |a|^2."""
    import scenegen as sg
    from oracle import geom, image
    s = sg.make_toy()
    s.V[:, 2] -= 1000.0  # move the scene far below the links
    g = geom.Geometry(s)
    rng = np.random.default_rng(4)
    pts = np.concatenate([rng.uniform(-50, 50, size=(6, 2)), rng.uniform(10, 60, size=(6, 1)),
                          rng.uniform(-80, 80, size=(6, 2))], 1)
    rx_z = 1.5
    prior = mlp.free_space_db(pts, 3.5e9, rx_z)
    from types import SimpleNamespace
    for k in range(len(pts)):
        dev = lambda p: SimpleNamespace(pos=tuple(p), yaw=0.0, pitch=0.0, roll=0.0, pattern=0)
        P = image.paths(g, dev(pts[k, :3]), [dev((pts[k, 3], pts[k, 4], rx_z))], [])[0]
        assert len(P) == 1 and P[0].faces == ()
        assert abs(10 * np.log10(abs(P[0].a) ** 2) - prior[k]) < 1e-9


def test_polynomial_gelu_of_map_inference_is_close_to_the_tanh_form():
    """The map-inference kernel evaluates GELU as x clamp(1/2 + u Q(u^2), 0, 1),
    u = clamp(x / 4, -1, 1); in exact arithmetic it stays within 2.5e-4 of the
    tanh form everywhere (coefficients as in the kernel)."""
    x = np.linspace(-12, 12, 48001)
    g = mlp.gelu_poly(x)
    assert np.max(np.abs(g - mlp.gelu(x))) < 2.5e-4 * np.maximum(1.0, np.abs(x)).max()
    assert np.max(np.abs(g - mlp.gelu(x))[np.abs(x) <= 4]) < 2.5e-4
    # outside |x| <= 4 it is exactly max(x, 0) (the clamp), as the tanh form is to 1e-3
    far = np.abs(x) >= 4
    assert np.array_equal(g[far], np.maximum(x[far], 0.0))


def test_half_precision_weights_round_to_nearest_and_keep_biases():
    theta, *_ = _problem(seed=4)
    r = mlp.round_weights_f16(theta)
    L0, L1 = mlp.unpack(theta), mlp.unpack(r)
    for li, ((W, b), (Wr, br)) in enumerate(zip(L0, L1)):
        assert np.array_equal(b, br)
        # each weight moves by at most half a unit in the last place of a half
        # (10 fraction bits; subnormals below 2^-14 have absolute spacing 2^-24)
        ulp = np.maximum(2.0 ** (np.floor(np.log2(np.maximum(np.abs(W), 2.0 ** -14))) - 10), 2.0 ** -24)
        sc = 0.25 if li == 0 else (4.0 if li == 4 else 1.0)
        assert np.all(np.abs(Wr - W) <= 0.5 * ulp / min(sc, 1.0) + 1e-18)
        assert np.all(np.float16(sc * Wr) == sc * Wr)
