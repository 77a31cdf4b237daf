"""GPU parity of the differentiable form (cfs_splat, cfs_splat_backward and
the torch.autograd wrapper) against the FP64 oracle.

Bars: density within 2e-5 of the density's maximum (FP32 weights, FP32
atomic order); gradient within 1e-4 relative L2 of the oracle's FP64 adjoint
for the same upstream gradient, and within 1e-3 of central finite
differences; gradient exactly zero at the target; checkpoints equal to the
plain chaos game's FP32 positions bit for bit; backward deterministic.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02226_amd import api as _api
    return _api


def _dev():
    return torch.device("cuda:0")


def gpu_forward(api, system, run, image, sigma=1.0, every=8):
    img = api.Image(image, device=_dev()).clear()
    N, T = run["n_points"], run["n_iters"]
    ckpt = torch.empty((api.n_checkpoints(T, every), N, 2), dtype=torch.float32, device=_dev())
    api.splat(system, run, img, sigma, ckpt=ckpt, ckpt_every=every)
    torch.cuda.synchronize()
    return img, ckpt


def theta_of(system):
    return np.concatenate([system["A"].reshape(-1, 4), system["b"]], axis=1).astype(np.float64)


@pytest.mark.parametrize("sigma", [1.0, 2.0])
def test_density_parity(api, orc, sigma):
    w = W.differentiable(n_points=1 << 16)
    img, _ = gpu_forward(api, w["system"], w["run"], w["image"], sigma)
    got = img.data.cpu().numpy().astype(np.float64)
    ref = orc.splat_gauss(w["system"], w["run"], w["image"], sigma)
    err = np.max(np.abs(got - ref)) / np.max(ref)
    print(f"density sigma={sigma}: max err / max = {err:.2e}, sums {got.sum():.6f} {ref.sum():.6f}")
    assert err < 2e-5
    assert abs(got.sum() - ref.sum()) / ref.sum() < 1e-5


# sigma 1 takes the 6-tap kernels, sigma in (1, 2.5] the 16-tap ones (15 or
# 16 candidate taps per axis, margins of TAPS - 1 pixels beside tile 0)
SIGMAS = [1.0, 1.01, 2.0, 2.5]


# below 1 px most of the 6 candidate taps per axis lie at distance R = 3
# sigma or more and take weight 0 (at 0.3 px one or two taps per axis remain)
@pytest.mark.parametrize("sigma", [0.3, 0.6] + SIGMAS)
def test_density_ragged_and_offimage(api, orc, sigma):
    # ragged image (not a multiple of the 32-pixel tile), window cutting the
    # attractor so that footprints straddle and leave the image; the
    # gradient through the same off-image footprints against the adjoint
    w = W.differentiable(n_points=3000, n_iters=21, burn_in=3)
    image = {"kind": "f32_density", "width": 77, "height": 45, "channels": 1,
             "lo": [0.1, 0.3], "hi": [0.8, 0.7]}
    img, ckpt = gpu_forward(api, w["system"], w["run"], image, sigma, every=5)
    got = img.data.cpu().numpy().astype(np.float64)
    ref = orc.splat_gauss(w["system"], w["run"], image, sigma)
    assert np.max(np.abs(got - ref)) / np.max(ref) < 2e-5
    G = np.random.default_rng(4).standard_normal((45, 77)).astype(np.float32)
    g = api.splat_backward(w["system"], w["run"], img, sigma, torch.from_numpy(G).to(_dev()),
                           ckpt, 5).cpu().numpy().astype(np.float64)
    gref = orc.splat_gauss_backward(w["system"], w["run"], image, sigma, G.astype(np.float64))
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    print(f"ragged sigma={sigma}: gradient rel L2 {rel:.2e}")
    assert rel < 1e-4, rel


def test_checkpoints_match_chaos_game(api):
    w = W.differentiable(n_points=5000, n_iters=32, burn_in=8)
    every = 8
    _, ckpt = gpu_forward(api, w["system"], w["run"], w["image"], 1.0, every)
    ck = ckpt.cpu().numpy()
    for j in range(ck.shape[0]):
        t = j * every
        if t == 0:
            continue
        img = api.Image({"kind": "u32_count", "width": 8, "height": 8, "channels": 1,
                         "lo": [0, 0], "hi": [1, 1]}, device=_dev()).clear()
        fin = torch.empty((5000, 2), dtype=torch.float32, device=_dev())
        api.chaos_game(w["system"], dict(w["run"], n_iters=t, burn_in=t), img, final=fin)
        assert np.array_equal(fin.cpu().numpy(), ck[j])


def _upstream(orc, w, sigma=1.0):
    D = orc.splat_gauss(w["system"], w["run"], w["image"], sigma)
    Dt = orc.splat_gauss(w["target_system"], w["run"], w["image"], sigma)
    return 2.0 * (D - Dt)


@pytest.mark.parametrize("sigma", SIGMAS)
def test_gradient_vs_oracle_adjoint(api, orc, sigma):
    w = W.differentiable(n_points=1 << 16)
    G = _upstream(orc, w, sigma).astype(np.float32)
    img, ckpt = gpu_forward(api, w["system"], w["run"], w["image"], sigma)
    g = api.splat_backward(w["system"], w["run"], img, sigma, torch.from_numpy(G).to(_dev()),
                           ckpt, 8).cpu().numpy().astype(np.float64)
    ref = orc.splat_gauss_backward(w["system"], w["run"], w["image"], sigma,
                                   G.astype(np.float64))
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    print(f"gradient vs oracle adjoint, sigma={sigma}: rel L2 {rel:.2e}")
    assert rel < 1e-4


def test_no_splats_gradient_zero(api):
    # burn_in == n_iters: nothing is splatted, the checkpoints are still
    # written (equal to the plain chaos game's positions) and the gradient
    # is exactly zero, also over a workspace and gradient full of NaNs
    w = W.differentiable(n_points=3000, n_iters=16, burn_in=16, side=64)
    img, ckpt = gpu_forward(api, w["system"], w["run"], w["image"], 1.0, 8)
    assert torch.count_nonzero(img.data).item() == 0
    fin = torch.empty((3000, 2), dtype=torch.float32, device=_dev())
    cimg = api.Image({"kind": "u32_count", "width": 8, "height": 8, "channels": 1,
                      "lo": [0, 0], "hi": [1, 1]}, device=_dev()).clear()
    api.chaos_game(w["system"], dict(w["run"], n_iters=8, burn_in=8), cimg, final=fin)
    assert torch.equal(ckpt[1], fin)
    G = torch.randn((64, 64), dtype=torch.float32, device=_dev())
    grad = torch.full((4, 6), float("nan"), dtype=torch.float32, device=_dev())
    ws = torch.full((1 << 16,), 255, dtype=torch.uint8, device=_dev())
    api.splat_backward(w["system"], w["run"], img, 1.0, G, ckpt, 8, grad=grad, workspace=ws)
    assert torch.count_nonzero(grad).item() == 0


def test_no_points_and_every_splat_off_the_image(api, orc):
    # no points: nothing is read or written, the gradient is exactly zero;
    # a window that misses the attractor: every splat is dropped (and
    # counted), the density stays zero and so does the gradient
    w = W.differentiable(n_points=4096, n_iters=12, burn_in=2, side=64)
    empty = dict(w["run"], n_points=0)
    img = api.Image(w["image"], device=_dev()).clear()
    ckpt = torch.empty((api.n_checkpoints(12, 4), 1, 2), dtype=torch.float32, device=_dev())
    api.splat(w["system"], empty, img, 1.0, ckpt=ckpt, ckpt_every=4)
    torch.cuda.synchronize()
    assert torch.count_nonzero(img.data).item() == 0 and img.dropped.item() == 0
    G = torch.randn((64, 64), dtype=torch.float32, device=_dev())
    g = api.splat_backward(w["system"], empty, img, 1.0, G, ckpt, 4)
    assert torch.count_nonzero(g).item() == 0
    far = dict(w["image"], lo=[5.0, 5.0], hi=[6.0, 6.0])
    img2, ck2 = gpu_forward(api, w["system"], w["run"], far, 1.0, 4)
    assert torch.count_nonzero(img2.data).item() == 0
    ref = orc.splat_gauss(w["system"], w["run"], far, 1.0)
    assert np.count_nonzero(ref) == 0
    assert img2.dropped.item() == 4096 * 10
    g2 = api.splat_backward(w["system"], w["run"], img2, 1.0, G, ck2, 4)
    assert torch.count_nonzero(g2).item() == 0


def test_gradient_vs_finite_differences(api, orc):
    # parameters with 12 fractional bits so that +-h (a power of two) is exact
    w = W.differentiable(n_points=2048, n_iters=16, burn_in=4, side=64)
    th = np.round(theta_of(w["system"]) * 2**12) / 2**12
    tt = np.round(theta_of(w["target_system"]) * 2**12) / 2**12
    sysd = api.theta_to_system(th)
    tgt = api.theta_to_system(tt)
    run, image = w["run"], w["image"]
    Dt = orc.splat_gauss(tgt, run, image, 1.0)
    D = orc.splat_gauss(sysd, run, image, 1.0)
    img, ckpt = gpu_forward(api, sysd, run, image)
    G = torch.from_numpy((2.0 * (D - Dt)).astype(np.float32)).to(_dev())
    g = api.splat_backward(sysd, run, img, 1.0, G, ckpt, 8).cpu().numpy().astype(np.float64)

    def loss(t):
        return orc.gauss_loss(api.theta_to_system(t), run, image, 1.0, Dt)[0]

    h = 2.0**-20
    fd = np.zeros_like(th)
    for i in range(th.shape[0]):
        for j in range(6):
            e = np.zeros_like(th)
            e[i, j] = h
            fd[i, j] = (loss(th + e) - loss(th - e)) / (2 * h)
    rel = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    print(f"gradient vs FD: rel L2 {rel:.2e}")
    assert rel < 1e-3


def test_gradient_zero_at_target_and_deterministic(api):
    w = W.differentiable(n_points=1 << 16)
    img, ckpt = gpu_forward(api, w["system"], w["run"], w["image"])
    zero = torch.zeros_like(img.data)
    g0 = api.splat_backward(w["system"], w["run"], img, 1.0, zero, ckpt, 8)
    assert torch.count_nonzero(g0).item() == 0
    G = torch.randn_like(img.data)
    g1 = api.splat_backward(w["system"], w["run"], img, 1.0, G, ckpt, 8).cpu()
    g2 = api.splat_backward(w["system"], w["run"], img, 1.0, G, ckpt, 8).cpu()
    assert torch.equal(g1, g2)


@pytest.mark.parametrize("every", [1, 3, 8, 16])
def test_checkpoint_interval_invariance(api, orc, every):
    w = W.differentiable(n_points=4096, n_iters=20, burn_in=5, side=128)
    G = np.random.default_rng(3).standard_normal((128, 128)).astype(np.float32)
    img, ckpt = gpu_forward(api, w["system"], w["run"], w["image"], 1.0, every)
    g = api.splat_backward(w["system"], w["run"], img, 1.0, torch.from_numpy(G).to(_dev()),
                           ckpt, every).cpu().numpy().astype(np.float64)
    ref = orc.splat_gauss_backward(w["system"], w["run"], w["image"], 1.0, G.astype(np.float64))
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-4


def test_unequal_probabilities_8_maps(api, orc):
    rng = np.random.default_rng(5)
    A, b = W.random_affine_maps(rng, 7)
    A, b = W.normalise_to_unit_square(A, b)
    prob = rng.dirichlet(np.ones(7))
    system = W._system(A, b, prob=prob)
    run = {"seed": 3, "instance": 1, "n_points": 8192, "point_offset": 100, "n_iters": 24,
           "burn_in": 6}
    image = {"kind": "f32_density", "width": 96, "height": 96, "channels": 1,
             "lo": [0, 0], "hi": [1, 1]}
    img, ckpt = gpu_forward(api, system, run, image, 1.0, 6)
    ref_D = orc.splat_gauss(system, run, image, 1.0)
    assert np.max(np.abs(img.data.cpu().numpy() - ref_D)) / ref_D.max() < 2e-5
    G = np.random.default_rng(1).standard_normal((96, 96)).astype(np.float32)
    g = api.splat_backward(system, run, img, 1.0, torch.from_numpy(G).to(_dev()), ckpt, 6)
    ref = orc.splat_gauss_backward(system, run, image, 1.0, G.astype(np.float64))
    assert np.linalg.norm(g.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-4


def test_concentrated_tile_parts(api, orc):
    # two maps contracting by 50 onto fixed points a few pixels apart: every
    # record lands in one or two tiles, which then take the most workgroups
    # per tile, each with an equal share of the chunks
    A = np.array([[[0.02, 0.0], [0.0, 0.02]]] * 2, dtype=np.float32)
    b = np.array([[0.49, 0.5], [0.5, 0.49]], dtype=np.float32)
    system = W._system(A, b)
    run = {"seed": 11, "instance": 0, "n_points": 1 << 16, "point_offset": 0, "n_iters": 20,
           "burn_in": 4}
    image = {"kind": "f32_density", "width": 256, "height": 256, "channels": 1,
             "lo": [0, 0], "hi": [1, 1]}
    img, ckpt = gpu_forward(api, system, run, image, 1.0, 4)
    ref_D = orc.splat_gauss(system, run, image, 1.0)
    got = img.data.cpu().numpy().astype(np.float64)
    assert np.count_nonzero(ref_D) < 200
    assert np.max(np.abs(got - ref_D)) / ref_D.max() < 2e-5
    yy, xx = np.mgrid[0:256, 0:256]
    G = (1.0 + xx / 256.0 + 2.0 * yy / 256.0).astype(np.float32)  # smooth: no cancellation
    g = api.splat_backward(system, run, img, 1.0, torch.from_numpy(G).to(_dev()), ckpt, 4)
    ref = orc.splat_gauss_backward(system, run, image, 1.0, G.astype(np.float64))
    assert np.linalg.norm(g.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-4


def test_long_runs_many_chunk_batches(api, orc):
    # 400 iterations of 2^14 points: dozens of flushes of 32 blocks, over a
    # thousand chunks, so a sparse tile's one or two workgroups walk its runs
    # in several batches of 256 (some runs empty), dense tiles' in one
    w = W.differentiable(n_points=1 << 14, n_iters=400, burn_in=8)
    img, ckpt = gpu_forward(api, w["system"], w["run"], w["image"], 1.0, 8)
    got = img.data.cpu().numpy().astype(np.float64)
    ref = orc.splat_gauss(w["system"], w["run"], w["image"], 1.0)
    assert np.max(np.abs(got - ref)) / np.max(ref) < 2e-5
    assert abs(got.sum() - ref.sum()) / ref.sum() < 1e-5
    G = _upstream(orc, w).astype(np.float32)
    g = api.splat_backward(w["system"], w["run"], img, 1.0, torch.from_numpy(G).to(_dev()),
                           ckpt, 8).cpu().numpy().astype(np.float64)
    ref_g = orc.splat_gauss_backward(w["system"], w["run"], w["image"], 1.0,
                                     G.astype(np.float64))
    assert np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g) < 1e-4


def test_density_many_tiles(api, orc):
    # 1440 x 1440 pixels: 2025 tiles of 32 x 32, fewer workgroups per tile
    w = W.differentiable(n_points=1 << 15, n_iters=16, burn_in=4)
    image = dict(w["image"], width=1440, height=1440)
    img, _ = gpu_forward(api, w["system"], w["run"], image, 1.0, 4)
    got = img.data.cpu().numpy().astype(np.float64)
    ref = orc.splat_gauss(w["system"], w["run"], image, 1.0)
    assert np.max(np.abs(got - ref)) / np.max(ref) < 2e-5
    assert abs(got.sum() - ref.sum()) / ref.sum() < 1e-5


def test_autograd_function(api, orc):
    from paper_2606_02226_amd.autograd import cfs_splat
    w = W.differentiable(n_points=1 << 14)
    th = torch.tensor(theta_of(w["system"]), dtype=torch.float32, device=_dev(),
                      requires_grad=True)
    target = torch.from_numpy(orc.splat_gauss(w["target_system"], w["run"], w["image"], 1.0)
                              .astype(np.float32)).to(_dev())
    D = cfs_splat(th, w["run"], w["image"], 1.0, 8)
    loss = ((D - target) ** 2).sum()
    loss.backward()
    G = (2.0 * (D.detach().double().cpu().numpy() - target.double().cpu().numpy()))
    ref = orc.splat_gauss_backward(w["system"], w["run"], w["image"], 1.0, G)
    rel = np.linalg.norm(th.grad.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert rel < 1e-4


def test_full_size_differentiable(api):
    """The differentiable configuration at full size (2^20 points x 32
    iterations, 512x512, sigma 1 px, checkpoints every 8): the density's mass
    matches the kernel's closed-form integral, and the gradient equals the
    sum of the gradients of 16 point-range slices (each oracle-checked size)."""
    w = W.differentiable()
    N = 1 << 20
    img, ckpt = gpu_forward(api, w["system"], w["run"], w["image"])
    D = img.data.double()
    ig = math.sqrt(2 * math.pi) * math.erf(3 / math.sqrt(2)) - 6 * math.exp(-4.5)
    assert abs(D.sum().item() / ig**2 - 1.0) < 1e-4
    G = torch.randn_like(img.data)
    g_full = api.splat_backward(w["system"], w["run"], img, 1.0, G, ckpt, 8).double().cpu()
    g_sum = torch.zeros_like(g_full)
    S = N // 16
    for s in range(16):
        run = dict(w["run"], n_points=S, point_offset=s * S)
        im, ck = gpu_forward(api, w["system"], run, w["image"])
        g_sum += api.splat_backward(w["system"], run, im, 1.0, G, ck, 8).double().cpu() * (S / N)
    rel = (torch.linalg.norm(g_full - g_sum) / torch.linalg.norm(g_full)).item()
    assert rel < 1e-5, rel
