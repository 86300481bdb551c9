"""Kernel-level parity: the HIP FFT/Green pipeline and the constitutive
kernels against the CPU oracle, element by element on seeded inputs."""
import numpy as np
import pytest

from oracle import fourier, green, tensor
from oracle.laws import PA66, Thermoelastic
from paper_2109_14403_amd import hom
from paper_2109_14403_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 16), (16, 24, 32), (48, 32, 24), (32, 64, 16)]   # (nz, ny, nx): several tiles, ragged tails
TOL = {hom.FP64: 1e-14, hom.FP32: 1e-6}   # measured: 8.2e-16 and 3.3e-7 at most


def oracle_apply(f, op, p0, p1, lengths):
    n = fourier.directions(f.shape[1:], lengths)
    F = fourier.fft3(f)
    if op == hom.OP_PROJECTOR:
        G = green.projector(F, n)
    elif op == hom.OP_GAMMA0:
        G = green.gamma_isotropic(F, n, p0, p1)
    elif op == hom.OP_GRAD_PROJECTOR:
        G = green.gradient_projector(F, n)
    else:
        G = green.gamma_conduction(F, n, p0)
    return fourier.ifft3(G)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("precision", [hom.FP64, hom.FP32])
@pytest.mark.parametrize("op,p0,p1,C", [(hom.OP_PROJECTOR, 0, 0, 6), (hom.OP_GAMMA0, 1.3, 0.7, 6),
                                        (hom.OP_GRAD_PROJECTOR, 0, 0, 3), (hom.OP_GAMMA_CONDUCTION, 0.6, 0, 3)])
def test_green_pipeline_matches_oracle(shape, precision, op, p0, p1, C):
    rng = np.random.default_rng(hash((shape, op)) % 2**32)
    lengths = (1.0, 1.0, 1.0) if shape[0] == shape[2] else (1.0, 0.8, 1.3)
    f = rng.normal(size=(C,) + shape)
    f += 0.5  # nonzero mean: the zero frequency must be removed
    gpu = hom.apply_operator(f, op, p0, p1, precision=precision, lengths=lengths)
    ref = oracle_apply(f, op, p0, p1, lengths)
    err = np.abs(gpu - ref).max() / np.abs(ref).max()
    print(f"shape {shape} op {op} precision {precision}: max rel err {err:.2e}", flush=True)
    assert err <= TOL[precision]


# every long plan (96 = 12 x 8, 128 = 16 x 8, 256 = 16 x 16 points) on each pass (x, y and z)
LONG_SHAPES = [(16, 16, 256), (16, 256, 16), (256, 16, 16), (16, 96, 16), (128, 16, 16), (96, 16, 128),
               (16, 128, 96)]


@pytest.mark.parametrize("shape", LONG_SHAPES)
@pytest.mark.parametrize("precision", [hom.FP64, hom.FP32])
@pytest.mark.parametrize("op,p0,C", [(hom.OP_PROJECTOR, 0, 6), (hom.OP_GAMMA_CONDUCTION, 0.6, 3)])
def test_long_plans_match_oracle(shape, precision, op, p0, C):
    rng = np.random.default_rng(sum(shape) * 7 + op)
    lengths = (1.0, 0.9, 1.2)
    f = rng.normal(size=(C,) + shape) + 0.25
    gpu = hom.apply_operator(f, op, p0, 0.0, precision=precision, lengths=lengths)
    ref = oracle_apply(f, op, p0, 0.0, lengths)
    err = np.abs(gpu - ref).max() / np.abs(ref).max()
    print(f"long plan {shape} op {op} precision {precision}: max rel err {err:.2e}", flush=True)
    assert err <= TOL[precision]


# every y / z schedule the autotuner may pick (tile width x FFT plan variant)
# on every transform length, the length on the y and the z axis in turn
PLAN_SHAPES = [(16, 24, 16), (24, 16, 16), (32, 48, 16), (48, 32, 16), (64, 96, 16), (96, 64, 16),
               (128, 16, 24), (16, 128, 24), (256, 16, 16), (16, 256, 16)]


@pytest.mark.parametrize("shape", PLAN_SHAPES)
@pytest.mark.parametrize("precision", [hom.FP64, hom.FP32])
def test_every_schedule_matches_oracle(shape, precision):
    rng = np.random.default_rng(sum(shape) * 11 + precision)
    lengths = (1.1, 0.9, 1.0)
    for op, p0, C in ((hom.OP_PROJECTOR, 0, 6), (hom.OP_GAMMA_CONDUCTION, 0.6, 3)):
        f = rng.normal(size=(C,) + shape) + 0.25
        ref = oracle_apply(f, op, p0, 0.0, lengths)
        for sc in hom.SCHEDULES:
            try:
                gpu = hom.apply_operator(f, op, p0, 0.0, precision=precision, lengths=lengths, schedule=sc)
            except hom.HomError as e:  # a tile wider than the work-group limits allow on this grid
                assert e.code == hom.HOM_E_UNSUPPORTED
                continue
            err = np.abs(gpu - ref).max() / np.abs(ref).max()
            print(f"schedule {sc} {shape} op {op} precision {precision}: max rel err {err:.2e}", flush=True)
            assert err <= TOL[precision]


def test_schedule_argument_errors():
    f = np.zeros((6, 16, 16, 16))
    with pytest.raises(hom.HomError) as e:
        hom.apply_operator(f, hom.OP_PROJECTOR, schedule=5)
    assert e.value.code == hom.HOM_E_ARG


def test_projector_output_is_compatible_and_idempotent():
    rng = np.random.default_rng(1)
    f = rng.normal(size=(6, 16, 24, 32))
    once = hom.apply_operator(f, hom.OP_PROJECTOR)
    twice = hom.apply_operator(once, hom.OP_PROJECTOR)
    assert np.abs(twice - once).max() <= 1e-12 * np.abs(once).max()
    assert np.abs(once.reshape(6, -1).mean(axis=1)).max() < 1e-13


def random_pa66_points(law, m, rng):
    st = law.initial_state(m)
    st["ep"] = rng.uniform(0.0, 0.02, size=m)
    st["ep"][: m // 3] = 0.0
    st["evp"] = tensor.deviator(rng.normal(scale=2e-3, size=(6, m)))
    st["ev"] = rng.normal(scale=2e-3, size=(law.N, 6, m))
    eps_n = rng.normal(scale=3e-3, size=(6, m))
    eps = eps_n + rng.normal(size=(6, m)) * np.logspace(-5, -1.5, m)[None]
    return st, eps, eps_n


def flat_state(st):
    return np.concatenate([st["ep"][None], st["evp"], st["ev"].reshape(-1, st["ep"].size)])


@pytest.mark.parametrize("theta,dt", [(293.15, 2.0), (333.15, 0.8), (373.15, 0.006), (300.0, 6.0)])
def test_pa66_kernel_matches_oracle(theta, dt):
    p = W.pa66()
    law = PA66(p)
    rng = np.random.default_rng(int(theta * 10))
    m = 3000
    st, eps, eps_n = random_pa66_points(law, m, rng)
    ref = law.update(eps, eps_n, st, theta, dt)
    out = hom.eval_law(p, eps, eps_n, flat_state(st), theta, dt, commit=True)
    scale = np.abs(ref["sigma"]).max(axis=0)
    assert (np.abs(out["sigma"] - ref["sigma"]).max(axis=0) <= 1e-10 * scale + 1e-12).all()
    # tangent K3 P1 + a P2 + b N N against the oracle's full matrix
    T = ref["tangent"]
    K3 = np.einsum("a,abk,b->k", tensor.IDENTITY2, T, tensor.IDENTITY2) / 3.0
    Tg = (K3[None, None] * tensor.P1[:, :, None] + out["ab"][0][None, None] * tensor.P2[:, :, None]
          + out["ab"][1][None, None] * np.einsum("ak,bk->abk", out["nd"], out["nd"]))
    tscale = np.abs(T).max(axis=(0, 1))
    assert (np.abs(Tg - T).max(axis=(0, 1)) <= 1e-8 * tscale).all()
    assert np.allclose(out["state"], flat_state(ref["state"]), rtol=1e-10, atol=1e-14)
    dscale = np.maximum(np.abs(ref["dissipation"]), 1e-6)
    assert (np.abs(out["dissipation"] - ref["dissipation"]) <= 1e-9 * dscale).all()
    cscale = np.maximum(np.abs(ref["coupling"]), 1e-6)
    assert (np.abs(out["coupling"] - ref["coupling"]) <= 1e-9 * cscale).all()
    assert (out["dissipation"] >= 0).all()
    assert (ref["delta"] > 0).any() and (ref["delta"] == 0).any()


def test_thermoelastic_kernel_matches_oracle():
    p = W.e_glass()
    law = Thermoelastic(p)
    rng = np.random.default_rng(5)
    eps_n = rng.normal(scale=1e-3, size=(6, 500))
    eps = eps_n + rng.normal(scale=1e-3, size=(6, 500))
    out = hom.eval_law(p, eps, eps_n, None, 320.0, 0.5, commit=True)
    assert np.allclose(out["sigma"], law.stress(eps, 320.0), rtol=1e-12, atol=1e-9)
    assert np.allclose(out["coupling"], law.coupling(eps, eps_n, 320.0, 0.5), rtol=1e-12)
    assert np.all(out["dissipation"] == 0.0)
    K, G = tensor.bulk_shear(p["E"], p["nu"])
    assert np.allclose(out["ab"][0], 2 * G) and np.all(out["ab"][1] == 0)
