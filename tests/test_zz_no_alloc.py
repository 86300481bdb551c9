"""The allocation-free ensemble inference (hom_mlp_ensemble_infer_static)
against the allocating entry point (hom_mlp_ensemble_infer) through the C ABI:
identical outputs on two calls in a row, the second with fewer rows, and a
request beyond the static array rejected before anything is launched."""
import numpy as np
import pytest
import torch

from paper_2109_14403_amd import hom

pytestmark = pytest.mark.gpu


def _nets(count, n_in=32, n_out=10):
    rng = np.random.default_rng(77)
    nets = []
    for s in range(count):
        net = hom.MLP(n_in, n_out, seed=100 + s)
        net.set_scaling(rng.normal(size=n_in), rng.uniform(0.5, 2.0, size=n_in), rng.normal(size=n_out),
                        rng.uniform(1.0, 3.0, size=n_out))
        nets.append(net)
    return nets


def test_static_ensemble_equals_allocating_entry_point():
    nets = _nets(3)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(5000, 32)).astype(np.float32)
    thr = None
    for n in (5000, 1234):            # the second call is smaller: stale rows of the first must not leak in
        x = torch.as_tensor(X[:n], device="cuda")
        y0, s0, a0 = hom.mlp_ensemble_infer(nets, x, 0.0, 1.0)
        torch.cuda.synchronize()
        if thr is None:
            thr = float(np.median(s0.cpu().numpy()))
        y0, s0, a0 = hom.mlp_ensemble_infer(nets, x, thr, 1.0)
        y1 = torch.full((n, 10), float("nan"), dtype=torch.float32, device="cuda")
        s1 = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        a1 = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        hom.mlp_ensemble_infer_static(nets, x, thr, 1.0, y1, s1, a1)
        torch.cuda.synchronize()
        print(f"static ensemble, {n} rows: accepted {a1.float().mean().item():.3f}", flush=True)
        assert torch.equal(y0, y1) and torch.equal(s0, s1) and torch.equal(a0, a1)
        acc = a1.cpu().numpy()
        assert acc.min() == 0 and acc.max() == 1


def test_static_ensemble_rejects_oversize_request():
    nets = _nets(2)
    n = hom.STATIC_SCRATCH_FLOATS // (2 * 10) + 1
    x = torch.zeros((n, 32), dtype=torch.float32, device="cuda")
    y = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    s = torch.empty((n,), dtype=torch.float32, device="cuda")
    a = torch.empty((n,), dtype=torch.uint8, device="cuda")
    with pytest.raises(hom.HomError) as e:
        hom.mlp_ensemble_infer_static(nets, x, 0.1, 1.0, y, s, a)
    assert e.value.code == hom.HOM_E_ARG and "static scratch" in str(e.value)
    # an empty request is a no-op
    hom.mlp_ensemble_infer_static(nets, x[:0], 0.1, 1.0, y[:0], s[:0], a[:0])
