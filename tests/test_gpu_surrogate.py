"""Surrogate with FFT fallback, end to end on a small training set.

Training rows come from the batched FFT solver on the fixed 32^3 sphere
microstructure; the checks are that the trained network improves on its own
fixed skip (the network is worth running), that acceptance is decided by the
spread exactly as documented, and that the calibrated threshold keeps every
accepted validation row within the target while rejected rows go to the FFT
solver (their error is then zero).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2109_14403_amd import hom  # noqa: E402
from paper_2109_14403_amd import surrogate as S  # noqa: E402

pytestmark = pytest.mark.gpu

HISTORIES = 800
TRAIN = 640


@pytest.fixture(scope="module")
def trained():
    img, _ = S.microstructure()
    hist = S.histories(HISTORIES, seed=21)
    sol = S.solve_histories(img, hist, chunk=HISTORIES)
    assert (sol["status"] == hom.HOM_OK).all()
    X, Y, den, hid = S.features(hist, sol)
    tr = hid < TRAIN
    sur = S.Surrogate()
    losses = sur.fit(X[tr], Y[tr], epochs=60, batch=256, lr=2e-3)
    return sur, losses, X, Y, den, tr


def _infer(sur, X):
    y, spread, acc = sur.infer(torch.as_tensor(X, device="cuda"))
    torch.cuda.synchronize()
    return y.cpu().numpy(), spread.cpu().numpy(), acc.cpu().numpy().astype(bool)


def test_training_loss_decreases(trained):
    _, losses, *_ = trained
    for L in losses:
        assert np.all(np.isfinite(L))
        assert L[-1] < 0.5 * L[0]


def test_network_beats_skip_only(trained):
    sur, _, X, Y, den, tr = trained
    y, _, _ = _infer(sur, X[~tr])
    err = S.stress_errors(y, Y[~tr], den[~tr])
    eskip = S.stress_errors(sur.skip_only(X[~tr]), Y[~tr], den[~tr])
    print(f"held-out median stress error: network {np.median(err):.3e}, skip only {np.median(eskip):.3e}")
    assert np.median(err) < np.median(eskip)


def test_mean_and_spread_definition(trained):
    """y is the ensemble mean; the spread is the RMS pairwise distance of the
    stress outputs over max(|mean stress|, floor)."""
    sur, _, X, _, _, tr = trained
    Xv = X[~tr][:1000]
    y, spread, _ = _infer(sur, Xv)
    ys = [net.forward(Xv) for net in sur.nets]
    M = len(ys)
    assert M >= 3
    ym = np.mean(ys, axis=0)
    np.testing.assert_allclose(y, ym, rtol=1e-6, atol=1e-6)
    pair = sum(np.sum((ys[a][:, :6] - ys[b][:, :6]) ** 2, axis=1) for a in range(M) for b in range(a + 1, M))
    rms = np.sqrt(pair / (M * (M - 1) / 2))
    m = np.maximum(np.linalg.norm(ym[:, :6], axis=1), sur.floor)
    np.testing.assert_allclose(spread, rms / m, rtol=1e-4, atol=1e-7)


def test_two_network_ensemble_is_the_pair_rule(trained):
    sur, _, X, _, _, tr = trained
    xd = torch.as_tensor(X[~tr][:777], device="cuda")
    yn, sn, an = hom.mlp_ensemble_infer(sur.nets[:2], xd, 0.01, sur.floor)
    torch.cuda.synchronize()
    ya, yb = sur.nets[0].forward(X[~tr][:777]), sur.nets[1].forward(X[~tr][:777])
    d = np.linalg.norm(ya[:, :6] - yb[:, :6], axis=1)
    m = np.maximum(np.linalg.norm(0.5 * (ya + yb)[:, :6], axis=1), sur.floor)
    np.testing.assert_allclose(yn.cpu().numpy(), 0.5 * (ya + yb), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(sn.cpu().numpy(), d / m, rtol=1e-4, atol=1e-7)
    near = np.abs(d / m - 0.01) < 1e-6      # ties at the threshold may round either way
    np.testing.assert_array_equal(an.cpu().numpy()[~near], (d / m <= 0.01)[~near])


def test_calibrated_acceptance_and_fallback(trained):
    sur, _, X, Y, den, tr = trained
    target = 1e-2
    info = sur.calibrate(X[~tr], Y[~tr], den[~tr], target=target, quantile=1.0)
    y, spread, acc = _infer(sur, X[~tr])
    np.testing.assert_array_equal(acc, spread <= sur.threshold)
    err = S.stress_errors(y, Y[~tr], den[~tr])
    assert acc.mean() == pytest.approx(info["accepted"])
    assert acc.any(), "no validation row accepted at a 1e-2 target"
    assert err[acc].max() <= target
    # rejected rows are answered by the FFT solver: the combined answer meets the target everywhere
    combined = np.where(acc[:, None], y, Y[~tr])
    assert S.stress_errors(combined, Y[~tr], den[~tr]).max() <= target


def test_negative_threshold_rejects_all(trained):
    sur, _, X, _, _, tr = trained
    saved = sur.threshold
    try:
        sur.threshold = -1.0
        _, _, acc = _infer(sur, X[~tr][:512])
        assert not acc.any()
    finally:
        sur.threshold = saved
