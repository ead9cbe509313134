"""Pin of the FP64 reference network used to check the GPU training kernels: its gradient
against central finite differences of its loss, for random parameters and inputs."""
import numpy as np

from oracle import mlp


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = rng.normal(0.0, 0.3, mlp.N_PARAMS)
    x = np.column_stack([rng.uniform(-1, 1, 40), rng.uniform(-1, 1, 40), rng.choice([-1.0, 1.0], 40)])
    t = rng.normal(0.0, 1.0, 40)
    L, g = mlp.loss_and_grad(theta, x, t)
    assert np.isfinite(L) and g.shape == (mlp.N_PARAMS,)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [0, 191, 192, 12736, 12800]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, x, t)[0] - mlp.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mlp_layout():
    d = {name: np.full(shp, k, dtype=float) for k, (name, shp) in enumerate(mlp.SHAPES)}
    theta = mlp.pack(d)
    assert theta.size == mlp.N_PARAMS == 12801
    # offsets of the flat layout: W1 0, b1 192, W2 256, b2 4352, W3 4416, ..., W5 12736, b5 12800
    assert theta[191] == 0 and theta[192] == 1 and theta[256] == 2 and theta[4352] == 3
    assert theta[12736] == 8 and theta[12800] == 9
