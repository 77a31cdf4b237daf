"""Pins of the oracle's Gaussian soft splat and its adjoint.

 - mass: averaged over splats whose pixel offsets are spread uniformly, the
   weight of one splat is (integral of g)^2 with
   integral g = sqrt(2 pi) erf(3 / sqrt 2) sigma - 6 sigma exp(-9/2);
 - the adjoint gradient equals central finite differences of the FP64 loss
   (h and 2h, Richardson-consistent);
 - at the target parameters the gradient is exactly zero.
"""
import math

import numpy as np
import pytest

import workloads as W


def small_problem(n_points=256, side=64, n_iters=16, burn_in=4):
    w = W.differentiable(n_points=n_points, n_iters=n_iters, burn_in=burn_in,
                         side=side)
    return w


def test_density_mass_closed_form(orc):
    w = small_problem(n_points=4096, side=256)
    # keep every splat away from the border so that no tap is cut off
    image = dict(w["image"], lo=[-0.1, -0.1], hi=[1.1, 1.1])
    D = orc.splat_gauss(w["system"], w["run"], image, 1.0)
    ig = math.sqrt(2 * math.pi) * math.erf(3 / math.sqrt(2)) - 6 * math.exp(-4.5)
    assert abs(D.sum() / ig**2 - 1.0) < 2e-4, D.sum() / ig**2


def test_density_sigma_scaling(orc):
    # with sigma = 2 px the integral scales by sigma^2 = 4
    w = small_problem(n_points=4096, side=256)
    image = dict(w["image"], lo=[-0.2, -0.2], hi=[1.2, 1.2])
    D = orc.splat_gauss(w["system"], w["run"], image, 2.0)
    ig = 2.0 * (math.sqrt(2 * math.pi) * math.erf(3 / math.sqrt(2)) - 6 * math.exp(-4.5))
    assert abs(D.sum() / ig**2 - 1.0) < 2e-4


def _theta(system):
    A = system["A"].astype(np.float64)
    b = system["b"].astype(np.float64)
    return np.concatenate([A.reshape(-1, 4), b], axis=1)  # [n][6]


def _system_from(theta, like):
    s = dict(like)
    s["A"] = theta[:, :4].reshape(-1, 2, 2).astype(np.float32)
    s["b"] = theta[:, 4:].astype(np.float32)
    return s


def test_adjoint_matches_finite_differences(orc):
    # Finite differences need parameter steps far below FP32 resolution, so the
    # step is applied through an exactly representable rescaling: parameters are
    # scaled to FP32 values with few mantissa bits, and h is a power of two.
    w = small_problem()
    theta = _theta(w["system"])
    theta = np.round(theta * 2**12) / 2**12  # 12 fractional bits: exact in FP32
    sys0 = _system_from(theta, w["system"])
    tgt = _system_from(np.round(_theta(w["target_system"]) * 2**12) / 2**12,
                       w["system"])
    run, image = w["run"], w["image"]
    D_t = orc.splat_gauss(tgt, run, image, 1.0)
    D = orc.splat_gauss(sys0, run, image, 1.0)
    G = 2.0 * (D - D_t)
    grad = orc.splat_gauss_backward(sys0, run, image, 1.0, G)

    def loss(th):
        return orc.gauss_loss(_system_from(th, w["system"]), run, image, 1.0, D_t)[0]

    h = 2.0**-20  # representable offset on top of 12-bit values (FP32 has 24)
    fd = np.zeros_like(theta)
    fd2 = np.zeros_like(theta)
    for i in range(theta.shape[0]):
        for j in range(6):
            e = np.zeros_like(theta)
            e[i, j] = h
            fd[i, j] = (loss(theta + e) - loss(theta - e)) / (2 * h)
            fd2[i, j] = (loss(theta + 2 * e) - loss(theta - 2 * e)) / (4 * h)
    rel = np.linalg.norm(grad - fd) / np.linalg.norm(fd)
    rel2 = np.linalg.norm(fd2 - fd) / np.linalg.norm(fd)
    assert rel2 < 1e-3, rel2  # the step is in the smooth regime
    assert rel < 1e-4, rel


def test_gradient_zero_at_target(orc):
    w = small_problem()
    run, image = w["run"], w["image"]
    D = orc.splat_gauss(w["system"], run, image, 1.0)
    grad = orc.splat_gauss_backward(w["system"], run, image, 1.0, 2.0 * (D - D))
    assert np.all(grad == 0.0)


def test_backward_linear_in_upstream(orc):
    w = small_problem()
    run, image = w["run"], w["image"]
    rng = np.random.default_rng(0)
    G1 = rng.standard_normal((64, 64))
    G2 = rng.standard_normal((64, 64))
    g1 = orc.splat_gauss_backward(w["system"], run, image, 1.0, G1)
    g2 = orc.splat_gauss_backward(w["system"], run, image, 1.0, G2)
    g12 = orc.splat_gauss_backward(w["system"], run, image, 1.0, G1 + 2 * G2)
    assert np.allclose(g12, g1 + 2 * g2, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("which", ["b", "A"])
def test_translation_gradient_closed_form(orc, which):
    # Chain rule: moving every map's offset (or a00) by the same h changes
    # the linear functional sum(G * D) by h times the sum over maps of the
    # per-map gradients.  Checked against a central difference of the oracle.
    w = small_problem()
    sys0 = dict(w["system"])
    a = 0.5
    sys0["A"] = np.stack([np.eye(2, dtype=np.float32) * a] * 4)
    run, image = w["run"], w["image"]
    rng = np.random.default_rng(4)
    G = rng.standard_normal((64, 64))
    grad = orc.splat_gauss_backward(sys0, run, image, 1.0, G)

    def lin(sysx):
        return float(np.sum(G * orc.splat_gauss(sysx, run, image, 1.0)))

    h = 2.0**-20  # b, a00 in [0.25, 1): the step is exact in FP32
    if which == "b":
        sp, sm = dict(sys0), dict(sys0)
        sp["b"] = (sys0["b"].astype(np.float64) + [h, 0]).astype(np.float32)
        sm["b"] = (sys0["b"].astype(np.float64) - [h, 0]).astype(np.float32)
        fd = (lin(sp) - lin(sm)) / (2 * h)
        got = grad[:, 4].sum()
    else:
        sp, sm = dict(sys0), dict(sys0)
        sp["A"] = (sys0["A"].astype(np.float64) + np.array([[h, 0], [0, 0]])).astype(np.float32)
        sm["A"] = (sys0["A"].astype(np.float64) - np.array([[h, 0], [0, 0]])).astype(np.float32)
        fd = (lin(sp) - lin(sm)) / (2 * h)
        got = grad[:, 0].sum()
    assert abs(got - fd) <= 1e-4 * max(1.0, abs(fd)), (got, fd)


def test_l2_loss_hand_values(orc):
    # L = sum (D - D*)^2 and dL/dD = 2 (D - D*), checked on values worked by hand
    loss, grad = orc.l2_loss(np.array([1.0, 2.0, 0.5], np.float32),
                             np.array([0.0, 3.0, 0.5], np.float32))
    assert loss == 2.0
    assert np.array_equal(grad, [2.0, -2.0, 0.0])
    loss, grad = orc.l2_loss(np.zeros(0, np.float32), np.zeros(0, np.float32))
    assert loss == 0.0 and grad.size == 0
