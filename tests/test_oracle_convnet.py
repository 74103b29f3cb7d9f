"""Pins of the warm-start network oracle: identity and strided-identity
kernels, brute-force central differences of a loss for every gradient, the
closed-form first Adam step, and exactness of the coarse-to-node
interpolation on constant and linear fields."""
import numpy as np
import pytest

import oracle.convnet as C


def test_identity_kernel_and_stride():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 6, 5, 4))
    w = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0
    assert np.allclose(C.conv3d_forward(x, w, None, (1, 1, 1), False), x)
    y = C.conv3d_forward(x, w, None, (2, 2, 1), False)
    assert y.shape == (2, 3, 3, 3, 4) and np.allclose(y, x[:, :, ::2, ::2, :])
    w1 = rng.standard_normal((4, 3, 1, 1, 1))
    assert np.allclose(C.conv3d_forward(x, w1, None, (1, 1, 1), False),
                       np.einsum("oc,ncdhw->nodhw", w1[..., 0, 0, 0], x))


@pytest.mark.parametrize("K,strides,relu", [(3, (1, 1, 1), False), (3, (2, 1, 2), True), (1, (1, 1, 1), True),
                                            (3, (3, 2, 2), True)])
def test_gradients_match_central_differences(K, strides, relu):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 2, 7, 5, 4))
    w = rng.standard_normal((3, 2, K, K, K))
    b = rng.standard_normal(3)
    t = rng.standard_normal(C.conv3d_forward(x, w, b, strides, relu).shape)

    def loss(x_, w_, b_):
        return C.mse(C.conv3d_forward(x_, w_, b_, strides, relu), t)[0]

    y = C.conv3d_forward(x, w, b, strides, relu)
    dy = C.mse(y, t)[1]
    dx, dw, db = C.conv3d_backward(x, w, y, dy, strides, relu)
    h = 1e-6
    for arr, grad, name in ((x, dx, "x"), (w, dw, "w"), (b, db, "b")):
        for idx in list(np.ndindex(arr.shape))[:: max(1, arr.size // 12)]:
            e = np.zeros_like(arr)
            e[idx] = h
            args = {"x": x, "w": w, "b": b}
            ap, am = dict(args), dict(args)
            ap[name] = arr + e
            am[name] = arr - e
            fd = (loss(ap["x"], ap["w"], ap["b"]) - loss(am["x"], am["w"], am["b"])) / (2 * h)
            assert fd == pytest.approx(grad[idx], rel=1e-5, abs=1e-8), (name, idx)


def test_adam_first_step_is_a_signed_lr_step():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = C.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 0.0, 1)
    assert np.allclose(p, -0.01 * np.sign(g))


def test_grid_to_nodes_constant_and_linear():
    base = np.full(9 * 7 * 5, 2.0)
    c = np.full((2, 3, 4), 0.25)
    assert np.allclose(C.grid_to_nodes(c, 9, 7, 5, base), 2.5)
    gx = 4
    lin = np.broadcast_to(np.arange(gx, dtype=float), (2, 3, gx)).copy()
    out = C.grid_to_nodes(lin, 17, 7, 5, np.ones(17 * 7 * 5)).reshape(5, 7, 17) - 1.0
    # node j at x-position u = j/16*4 - 1/2 cell units: linear in j between the outer centres
    u = np.arange(17) / 16 * 4 - 0.5
    assert np.allclose(out[0, 0], np.clip(u, 0, gx - 1))


def test_trace_features_pick_component_receiver_and_step():
    rng = np.random.default_rng(2)
    tr = rng.standard_normal((2, 11, 6, 3))
    f = C.trace_features(tr, np.array([4, 1]), 4, 1, 3, 2, 2.0)
    assert f[1, 2, 0] == 2.0 * tr[1, 7, 4, 2] and f[0, 3, 1] == 2.0 * tr[0, 10, 1, 2]
    assert C.trace_features(tr, np.array([0]), 5, 1, 3, 0, 1.0)[0, 4, 0] == 0.0


def test_bf16_rounding_matches_the_format():
    """Nearest-even rounding to 8 significant bits: exact BF16 values stay,
    halfway cases go to the even neighbour, the relative error is at most 2^-8."""
    from oracle.convnet import bf16_round
    assert bf16_round(np.float32(1.0)) == 1.0
    one_ulp = 2.0 ** -7                       # BF16 spacing at 1
    assert bf16_round(np.float32(1.0 + one_ulp / 2)) == 1.0            # tie -> even (1.0)
    assert bf16_round(np.float32(1.0 + 3 * one_ulp / 2)) == 1.0 + 2 * one_ulp   # tie -> even
    assert bf16_round(np.float32(1.0 + 0.6 * one_ulp)) == 1.0 + one_ulp
    x = np.random.default_rng(2).standard_normal(10000).astype(np.float32)
    r = bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    # rounded values have at most 8 significant bits
    m, _ = np.frexp(r)
    assert np.all(np.abs(m * 2 ** 8 - np.round(m * 2 ** 8)) == 0)
