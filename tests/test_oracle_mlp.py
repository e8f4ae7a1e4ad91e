"""Pins of the FP64 reference of the learned proposal (oracle/mlp_oracle.py),
CPU only: the back-propagated gradient against central finite differences (a
different method), closed forms at zero parameters and for Adam's first step,
the published SplitMix64 output, and properties of the leverage features."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo


def _rand_problem(seed, n=300):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mo.NPARAMS) * 0.3
    X = rng.standard_normal((n, mo.F))
    y = (rng.random(n) < 0.2).astype(np.float64)
    return p, X, y


@pytest.mark.parametrize("pw", [1.0, 3.0])
def test_gradient_matches_central_differences(pw):
    p, X, y = _rand_problem(1)
    g = mo.grad(p, X, y, pw)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mo.NPARAMS, 300, replace=False), np.arange(mo.P_B1, mo.P_W2),
                          [mo.P_B3]])
    h = 1e-6
    fd = np.empty(len(idx))
    for q, k in enumerate(idx):
        e = np.zeros(mo.NPARAMS)
        e[k] = h
        fd[q] = (mo.loss(p + e, X, y, pw) - mo.loss(p - e, X, y, pw)) / (2 * h)
    np.testing.assert_allclose(g[idx], fd, rtol=0, atol=1e-7 * max(1.0, np.abs(g).max()))


def test_zero_parameters_closed_form():
    # all parameters 0: every score is 0, softplus(0) = ln 2, dL/ds = (1 - y - pw y) / (2 N),
    # and only b3 has a nonzero gradient (the hidden units are exactly 0)
    _, X, y = _rand_problem(3)
    p = np.zeros(mo.NPARAMS)
    pw = 2.5
    assert mo.loss(p, X, y, pw) == pytest.approx(np.log(2.0) * np.mean(pw * y + 1.0 - y), rel=1e-15)
    g = mo.grad(p, X, y, pw)
    assert g[mo.P_B3] == pytest.approx(np.sum(1.0 - y - pw * y) / (2 * len(y)), rel=1e-14)
    g[mo.P_B3] = 0.0
    assert not g.any()


def test_adam_first_step_closed_form():
    # t = 1: m1/(1-b1) = g, m2/(1-b2) = g^2, so the step is lr g / (|g| + eps)
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    p1, m1, m2 = mo.adam(p, z, z, g, 1, 0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(m2, 0.001 * g * g, rtol=1e-12)  # 1 - 0.999 rounds


def test_splitmix64_published_output_and_gauss_moments():
    # SplitMix64 started from state 0 first outputs 0xe220a8397b1dcdaf
    assert mo._splitmix64(0) == 0xE220A8397B1DCDAF
    x = mo.gauss(12345, 40000)
    assert abs(x.mean()) < 0.02 and abs(x.var() - 1.0) < 0.03
    np.testing.assert_array_equal(mo.gauss(12345, 100), x[:100])  # a pure function of (seed, index)


def test_features_properties():
    rng = np.random.default_rng(5)
    m, n, r, w = 300, 200, 8, 64
    A = rng.standard_normal((m, 30)) @ rng.standard_normal((30, n))
    A[17] *= 50.0  # one dominant row: leverage near 1, top rank in every leaf
    Fe = mo.features(A, r, w, 99)
    b = n // w
    assert Fe.shape == (b * m, 4)
    f1 = Fe[:m, 1]
    lev = 2.0 ** f1 * (2 * r) / m
    assert lev.sum() == pytest.approx(2 * r, rel=1e-9)  # leverage sums to the sketch rank
    for k in range(b):
        blk = Fe[k * m:(k + 1) * m]
        c0, c1 = k * w, (n if k == b - 1 else (k + 1) * w)
        assert blk[:, 0].max() == 0.0 and (blk[:, 0] <= 0).all()
        assert np.argmax(blk[:, 0]) == 17
        # ridge leverage: sum_i lb_i = trace(G (G + lam I)^-1) = sum_j sig_j^2 / (sig_j^2 + lam),
        # from the block's singular values; every lb_i lies in [0, 1)
        lb = 2.0 ** blk[:, 2] * (c1 - c0) / m
        sig2 = np.linalg.svd(A[:, c0:c1], compute_uv=False) ** 2
        lam = 2.0 ** -20 * (A[:, c0:c1] ** 2).sum(axis=0).max()
        assert lb.sum() == pytest.approx((sig2 / (sig2 + lam)).sum(), rel=1e-9)
        assert ((lb >= 0) & (lb < 1)).all()
        assert lb[17] > 0.99 and blk[17, 3] < 2.0 / m  # the dominant row leads its leaf
        assert ((blk[:, 3] >= 0) & (blk[:, 3] < 1)).all()
    assert lev[17] > 0.99
