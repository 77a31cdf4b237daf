"""Fitting loop on top of the differentiable form: starting from perturbed
parameters, gradient steps through cfs_splat_backward recover the target
system (common random numbers make the loss zero at the target)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_fit_recovers_target():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02226_amd import api
    from paper_2606_02226_amd.fit import fit
    w = W.differentiable(n_points=1 << 15, side=128)
    run, image = w["run"], w["image"]
    theta_t = np.concatenate([w["target_system"]["A"].reshape(-1, 4),
                              w["target_system"]["b"]], axis=1).astype(np.float64)
    theta_0 = np.concatenate([w["system"]["A"].reshape(-1, 4), w["system"]["b"]],
                             axis=1).astype(np.float64)
    img = api.Image(image, device="cuda").clear()
    api.splat(api.theta_to_system(theta_t.astype(np.float32)), run, img, 1.0)
    target = img.data.clone()
    theta, hist = fit(theta_0, target, run, image, steps=150, lr=2e-3)
    err0 = np.linalg.norm(theta_0 - theta_t)
    err1 = np.linalg.norm(theta - theta_t)
    print(f"fit: loss {hist[0]:.3e} -> {hist[-1]:.3e}, |theta - theta*| {err0:.3e} -> {err1:.3e}")
    assert hist[-1] < 0.05 * hist[0]
    assert err1 < 0.3 * err0


@pytest.mark.parametrize("n", [0, 1, 1000, 512 * 512, 3_000_017])
def test_l2_loss_parity(n):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle as orc
    from paper_2606_02226_amd import api
    rng = np.random.default_rng(n)
    d = rng.random(n, dtype=np.float32) * 1e-3
    t = rng.random(n, dtype=np.float32) * 1e-3
    loss, grad = api.l2_loss(torch.from_numpy(d).cuda(), torch.from_numpy(t).cuda())
    ref_loss, ref_grad = orc.l2_loss(d, t)
    got = float(loss.item())
    assert abs(got - ref_loss) <= 1e-12 * max(ref_loss, 1e-300)
    g = grad.cpu().numpy().astype(np.float64)
    # one rounding of 2 (D - D*) to FP32
    assert np.all(np.abs(g - ref_grad) <= np.abs(ref_grad) * 2.0 ** -24)
    loss2, _ = api.l2_loss(torch.from_numpy(d).cuda(), torch.from_numpy(t).cuda())
    assert float(loss2.item()) == got          # fixed reduction order
