"""Host logic of the surrogate (no GPU): the library's input rows
(hom_surrogate_features) against the layout include/hom.h documents, built
here independently from the histories and their answers."""
import numpy as np
import pytest

from paper_2109_14403_amd import hom

SQ2 = np.sqrt(2.0)
W = np.array([1, 1, 1, SQ2, SQ2, SQ2])


def fake_answers(rng, count, steps):
    f = np.zeros((count, steps), dtype=hom.RESULT_DTYPE)
    f["stress"] = rng.normal(scale=20.0, size=(count, steps, 6))
    f["heat_flux"] = rng.normal(size=(count, steps, 3))
    f["dissipation"] = rng.uniform(0.0, 0.01, size=(count, steps))
    return f


def expected_rows(strain, theta, grad, dt, fft, theta_init):
    count, steps = theta.shape
    X = np.zeros((count, steps, 32))
    Y = np.zeros((count, steps, 10))
    den = np.zeros((count, steps))
    for h in range(count):
        sig = fft["stress"][h] * W
        den[h] = np.linalg.norm(sig, axis=1).max()
        for k in range(steps):
            X[h, k, 0:6] = strain[h, k] * W
            X[h, k, 6] = theta[h, k]
            X[h, k, 7] = np.log10(dt[h, k])
            if k >= 1:
                X[h, k, 8:14] = strain[h, k - 1] * W
                X[h, k, 14:20] = sig[k - 1]
            if k >= 2:
                X[h, k, 20:26] = strain[h, k - 2] * W
            X[h, k, 26] = theta[h, k - 1] if k >= 1 else theta_init
            X[h, k, 27] = fft["dissipation"][h, k - 1] if k >= 1 else 0.0
            X[h, k, 28] = sum(fft["dissipation"][h, j] * dt[h, j] for j in range(k))
            X[h, k, 29:32] = grad[h, k]
            Y[h, k, 0:6] = sig[k]
            Y[h, k, 6:9] = fft["heat_flux"][h, k]
            Y[h, k, 9] = fft["dissipation"][h, k]
    return X.reshape(-1, 32), Y.reshape(-1, 10), den.reshape(-1)


def test_feature_rows_follow_the_documented_layout():
    rng = np.random.default_rng(4)
    count, steps = 3, 5
    strain = rng.normal(scale=5e-3, size=(count, steps, 6))
    theta = 293.15 + rng.uniform(0, 80, size=(count, steps))
    grad = rng.normal(size=(count, steps, 3))
    dt = np.exp(rng.uniform(-5, 1.5, size=(count, steps)))
    fft = fake_answers(rng, count, steps)
    X, Y, den = hom.surrogate_features(strain, theta, grad, dt, fft, theta_init=290.0)
    Xe, Ye, de = expected_rows(strain, theta, grad, dt, fft, 290.0)
    np.testing.assert_allclose(X, Xe.astype(np.float32), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(Y, Ye.astype(np.float32), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(den, de, rtol=1e-14)


def test_per_history_theta_dt_and_grad_broadcast():
    rng = np.random.default_rng(8)
    count, steps = 2, 3
    strain = rng.normal(scale=5e-3, size=(count, steps, 6))
    theta = 300.0 + rng.uniform(0, 10, size=count)
    grad = rng.normal(size=(count, 3))
    dt = np.array([0.5, 2.0])
    fft = fake_answers(rng, count, steps)
    X, _, _ = hom.surrogate_features(strain, theta, grad, dt, fft)
    Xe, _, _ = expected_rows(strain, np.repeat(theta[:, None], steps, 1), np.repeat(grad[:, None], steps, 1),
                             np.repeat(dt[:, None], steps, 1), fft, 293.15)
    np.testing.assert_allclose(X, Xe.astype(np.float32), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("bad", ["dt", "theta"])
def test_feature_rows_reject_bad_histories(bad):
    rng = np.random.default_rng(9)
    strain = rng.normal(size=(2, 2, 6))
    theta = np.full((2, 2), 300.0)
    dt = np.ones((2, 2))
    if bad == "dt":
        dt[1, 1] = 0.0
    else:
        theta[0, 1] = -1.0
    with pytest.raises(hom.HomError) as e:
        hom.surrogate_features(strain, theta, np.zeros((2, 2, 3)), dt, fake_answers(rng, 2, 2))
    assert e.value.code == hom.HOM_E_ARG
