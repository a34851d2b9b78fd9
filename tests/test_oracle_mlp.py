"""Pins of the cost-model oracle: forward pass against a closed form, the
analytic gradient against central finite differences, and the FP32 forward
against the FP64 one."""
import numpy as np

import synth

P = 4803
H, F = 64, 6
OW1, OB1 = 0, 384
OW2, OB2 = 448, 4544
OW3, OB3 = 4608, 4800


def seeded_weights(seed, scale=0.3):
    return (synth.uniform(seed, 9, P) * 2 - 1) * scale


def seeded_records(seed, B):
    feat = (synth.uniform(seed, 10, B * F) * 2 - 1).reshape(B, F)
    kind = np.floor(synth.uniform(seed, 11, B) * 3).astype(np.int32)
    tgt = synth.uniform(seed, 12, B) * 4 - 1
    return feat, kind, tgt


def test_forward_closed_form(ora):
    # a network that copies f0 through one unit: h1_0 = relu(f0), h2_0 = relu(h1_0), y_j = (j+1) h2_0 + b
    w = np.zeros(P)
    w[OW1 + 0 * F + 0] = 1.0
    w[OW2 + 0 * H + 0] = 1.0
    for j in range(3):
        w[OW3 + j * H + 0] = j + 1.0
        w[OB3 + j] = -0.5 * j
    for f0 in (-0.7, 0.0, 0.3, 2.5):
        f = np.array([f0, 1, 1, 1, 1, 1.0])
        y = ora.mlp_forward(w, f)
        r = max(f0, 0.0)
        assert np.allclose(y, [r, 2 * r - 0.5, 3 * r - 1.0], rtol=0, atol=1e-15)


def test_zero_loss_at_own_outputs(ora):
    w = seeded_weights(1)
    feat, kind, _ = seeded_records(2, 8)
    tgt = np.array([ora.mlp_forward(w, feat[r])[kind[r]] for r in range(8)])
    loss, g = ora.mlp_loss_grad(w, feat, kind, tgt)
    assert loss < 1e-28 and np.abs(g).max() < 1e-13


def test_gradient_matches_finite_differences(ora):
    w = seeded_weights(3)
    feat, kind, tgt = seeded_records(4, 12)
    loss, g = ora.mlp_loss_grad(w, feat, kind, tgt)
    idx = np.concatenate([np.arange(OW1, OW1 + 20), np.arange(OB1, OB1 + 10), np.arange(OW2, OW2 + 40, 3),
                          np.arange(OB2, OB2 + 10), np.arange(OW3, OW3 + 192, 7), np.arange(OB3, OB3 + 3)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (ora.mlp_loss_grad(wp, feat, kind, tgt)[0] - ora.mlp_loss_grad(wm, feat, kind, tgt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-8, i


def test_loss_is_mean_squared_error(ora):
    w = seeded_weights(5)
    feat, kind, tgt = seeded_records(6, 9)
    y = np.array([ora.mlp_forward(w, feat[r]) for r in range(9)])
    ref = np.mean((y[np.arange(9), kind] - tgt) ** 2)
    loss, _ = ora.mlp_loss_grad(w, feat, kind, tgt)
    assert abs(loss - ref) < 1e-14 * max(1.0, ref)


def _grid_features(p, theta):
    """The quantised feature grid of the choice table, [9,81,81,4,6], FP64."""
    dl, bt, bs, bq = np.meshgrid(np.arange(-4, 5), np.arange(81), np.arange(81), np.arange(4), indexing="ij")
    f = np.stack([dl / 2.0, bt / 4.0 / 8.0, bs / 4.0 / 8.0, np.full(dl.shape, p / 10.0), (bq + 0.5) / 4.0,
                  np.full(dl.shape, theta)], axis=-1)
    return f


def _np_forward(w, f, dtype):
    """The network as three library matrix products in `dtype`."""
    w = np.asarray(w, dtype)
    f = np.asarray(f, dtype).reshape(-1, F)
    W1, b1 = w[OW1:OB1].reshape(H, F), w[OB1:OW2]
    W2, b2 = w[OW2:OB2].reshape(H, H), w[OB2:OW3]
    W3, b3 = w[OW3:OB3].reshape(3, H), w[OB3:OB3 + 3]
    h1 = np.maximum(f @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    return h2 @ W3.T + b3


def test_table64_is_the_argmin_of_the_forward(ora):
    w = seeded_weights(9).astype(np.float32).astype(np.float64)
    tab, mar, bnd = ora.mlp_table64(w, 10, 0.4)
    assert tab.shape == (9, 81, 81, 4) and set(np.unique(tab)) <= {0, 1, 2}
    y = _np_forward(w, _grid_features(10, 0.4), np.float64).reshape(9, 81, 81, 4, 3)
    ys = np.sort(y, axis=-1)
    clear = (ys[..., 1] - ys[..., 0]) > 1e-12
    assert np.array_equal(tab[clear], np.argmin(y, axis=-1)[clear])
    assert np.allclose(mar, ys[..., 1] - ys[..., 0], rtol=0, atol=1e-12)
    # spot checks through the oracle's own scalar forward
    for (dl, bt, bs, bq) in [(0, 0, 0, 0), (8, 80, 3, 3), (4, 17, 40, 2), (2, 60, 60, 1)]:
        f = np.array([(dl - 4) / 2, bt / 4 / 8, bs / 4 / 8, 1.0, (bq + 0.5) / 4, 0.4])
        assert tab[dl, bt, bs, bq] == int(np.argmin(ora.mlp_forward(w, f)))


def test_fp32_error_bound_holds(ora):
    """An FP32 evaluation (library matrix products, features rounded to FP32)
    stays within the oracle's bound of the FP64 outputs everywhere, and the
    bound is tight enough to decide nearly every entry."""
    for seed, p, theta in ((9, 10, 0.4), (31, 8, 0.5)):
        w = seeded_weights(seed).astype(np.float32)
        tab, mar, bnd = ora.mlp_table64(w, p, theta)
        f = _grid_features(p, theta)
        y64 = _np_forward(w.astype(np.float64), f, np.float64).reshape(9, 81, 81, 4, 3)
        y32 = _np_forward(w, f.astype(np.float32), np.float32).astype(np.float64).reshape(9, 81, 81, 4, 3)
        err = np.abs(y32 - y64).max(axis=-1)
        assert np.all(err <= bnd), float((err / bnd).max())
        assert np.median(bnd) < 1e-3
        decided = mar > 2 * bnd
        assert decided.mean() > 0.99
        assert np.array_equal(np.argmin(y32, axis=-1)[decided], tab[decided])
