"""GPU parity of the surrogate-network kernels (through the C ABI) against the FP64
reference oracle/mlp.py evaluated with the same BF16-rounded weights.

Tolerances: the kernels accumulate 256-term products in FP32 with FP32 GELU (the
matrix-core kernels take each FP32 activation as hi + lo BF16 parts, ~2^-17
relative), so values agree to ~1e-5 of their scale; parameter gradients to ~1e-4 of the
largest component of their block; Adam updates to FP32 rounding."""

import numpy as np
import pytest
import torch

from oracle import mlp
from synth.mlp_init import init_params
from paper_2407_11349_amd.surrogate import SurrogateNet, Standardiser, Surrogate, train

pytestmark = pytest.mark.gpu


def _data(B, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(B, 6)) * scale).astype(np.float32), rng.normal(size=B).astype(np.float32), \
        rng.normal(size=(B, 6)).astype(np.float32)


def _bf16_params(p32):
    return mlp.to_bf16(p32)


@pytest.mark.parametrize("B", [1, 8, 9, 16, 37, 300, 4099])
def test_forward_value_and_input_gradient(B):
    """Batches of up to 8 take the one-sample kernel, larger ones the matrix-core tiles of 16 samples
    (ragged last tile at 9, 37, 300 and 4099)."""
    p = init_params(11) * 2.0
    net = SurrogateNet(p)
    z, _, _ = _data(B, 1)
    f, gz = net.forward(torch.from_numpy(z))
    torch.cuda.synchronize()
    f_ref, gz_ref = mlp.forward(_bf16_params(p), z.astype(np.float64))
    np.testing.assert_allclose(f.cpu().numpy(), f_ref, rtol=1e-4, atol=2e-5 * np.abs(f_ref).max())
    np.testing.assert_allclose(gz.cpu().numpy(), gz_ref, rtol=1e-4, atol=2e-5 * np.abs(gz_ref).max())


@pytest.mark.parametrize("B", [1, 37, 64, 300])
def test_sobolev_loss_and_parameter_gradient(B):
    """Matrix-core training pass over ragged and whole 32-sample chunks of the batch."""
    p = init_params(12) * 2.0
    net = SurrogateNet(p)
    z, y, g = _data(B, 2)
    lam = 0.5
    loss, grad = net.loss_grad(torch.from_numpy(z), torch.from_numpy(y), torch.from_numpy(g), lam)
    torch.cuda.synchronize()
    loss_ref, grad_ref = mlp.sobolev_loss_and_grad(_bf16_params(p), z.astype(np.float64), y.astype(np.float64),
                                                   g.astype(np.float64), lam)
    assert float(loss.item()) == pytest.approx(loss_ref, rel=2e-5)
    grad = grad.cpu().numpy()
    for name, shp, off in mlp.layout():
        n = int(np.prod(shp))
        a, b = grad[off:off + n], grad_ref[off:off + n]
        np.testing.assert_allclose(a, b, rtol=1e-3, atol=1e-4 * np.abs(b).max(), err_msg=name)
    # deterministic: a second call gives the same bits
    _, grad2 = net.loss_grad(torch.from_numpy(z), torch.from_numpy(y), torch.from_numpy(g), lam)
    assert np.array_equal(grad2.cpu().numpy(), grad)


def test_adam_update_and_bf16_refresh():
    p = init_params(13)
    net = SurrogateNet(p)
    rng = np.random.default_rng(3)
    m = np.zeros(p.shape[0])
    v = np.zeros(p.shape[0])
    th = p.astype(np.float64)
    for step in (1, 2, 3):
        gr = rng.normal(size=p.shape[0]).astype(np.float32)
        net.adam_step(torch.from_numpy(gr).cuda(), step, 1e-3)
        th, m, v = mlp.adam_step(th, m, v, gr.astype(np.float64), step, 1e-3)
    got = net.params().cpu().numpy()
    np.testing.assert_allclose(got, th, rtol=1e-5, atol=1e-7)
    # the BF16 working copy follows the master weights: the forward pass matches the oracle on them
    z, _, _ = _data(5, 4)
    f, _ = net.forward(torch.from_numpy(z))
    f_ref, _ = mlp.forward(mlp.to_bf16(got), z.astype(np.float64))
    np.testing.assert_allclose(f.cpu().numpy(), f_ref, rtol=1e-4, atol=1e-5)


def test_training_fits_a_smooth_six_dimensional_function():
    """Adam on the Sobolev loss learns a correlated Gaussian log-density from (z, value,
    gradient) tuples; held-out value and gradient errors fall well below the data spread."""
    rng = np.random.default_rng(5)
    A = rng.normal(size=(6, 6))
    Q = A @ A.T / 6 + np.eye(6)
    c = rng.normal(size=6) * 0.3

    def target(x):
        d = x - c
        return -0.5 * np.einsum("bi,ij,bj->b", d, Q, d), -(d @ Q)

    x = rng.normal(size=(6000, 6))
    yv, gv = target(x)
    std = Standardiser.fit(x, yv)
    net = SurrogateNet(init_params(14))
    hist = train(net, std, x[:5000], yv[:5000], gv[:5000], lam=1.0, epochs=30, batch=250, lr=2e-3, seed=1)
    assert hist[-1] < 0.05 * hist[0]
    sur = Surrogate(net, std)
    yh, gh = sur.value_and_grad(x[5000:])
    yt, gt = yv[5000:], gv[5000:]
    assert np.sqrt(np.mean((yh - yt) ** 2)) < 0.05 * yt.std()
    assert np.sqrt(np.mean((gh - gt) ** 2)) < 0.1 * gt.std()


def test_training_up_to_one_offset_per_group():
    """Tuples in groups of 21, each group's values shifted by a large random offset (as a
    latent-location draw shifts the log-likelihood): trained with the groups, the network
    fits the function up to per-group offsets, and better than trained without them."""
    from paper_2407_11349_amd.surrogate import group_means

    rng = np.random.default_rng(9)
    A = rng.normal(size=(6, 6))
    Q = A @ A.T / 6 + np.eye(6)

    def target(x):
        return -0.5 * np.einsum("bi,ij,bj->b", x, Q, x), -(x @ Q)

    n_groups, per = 300, 21
    x = rng.normal(size=(n_groups * per, 6)) * 0.5
    groups = np.repeat(np.arange(n_groups), per)
    yv, gv = target(x)
    offsets = rng.normal(size=n_groups) * 30.0
    yn = yv + offsets[groups]
    tr = groups < 270
    te = ~tr

    def within_rmse(net, std):
        yh, _ = Surrogate(net, std).value_and_grad(x[te])
        e = yh - yv[te]
        g = groups[te] - 270
        return np.sqrt(np.mean((e - group_means(e, g)[g]) ** 2))

    spread = np.sqrt(np.mean((yv[te] - group_means(yv[te], groups[te] - 270)[groups[te] - 270]) ** 2))
    std_g = Standardiser.fit(x[tr], yn[tr], groups[tr])
    net_g = SurrogateNet(init_params(21))
    train(net_g, std_g, x[tr], yn[tr], gv[tr], lam=1.0, epochs=30, batch=256, lr=2e-3, seed=2, groups=groups[tr])
    std_p = Standardiser.fit(x[tr], yn[tr])
    net_p = SurrogateNet(init_params(21))
    train(net_p, std_p, x[tr], yn[tr], gv[tr], lam=1.0, epochs=30, batch=256, lr=2e-3, seed=2)
    e_g, e_p = within_rmse(net_g, std_g), within_rmse(net_p, std_p)
    print(f"within-group rmse: grouped {e_g:.3f}, plain {e_p:.3f}, spread {spread:.3f}", flush=True)
    assert e_g < 0.1 * spread
    assert e_g < e_p


def _std():
    return Standardiser(m_z=np.array([-0.1, 1.9, 2.0, -2.1, 3.3, -3.1]),
                        s_z=np.array([0.01, 0.02, 0.05, 0.03, 0.04, 0.08]), m_y=-5.4e5, s_y=4.0)


def test_fused_leapfrog_equals_host_leapfrog():
    """The one-kernel trajectory (hawkes_mlp_leapfrog) against the host leapfrog of the sampler
    layer driving the same network call by call: positions, momenta and gradients bitwise (the
    same FP64 operations in the same order, the same network arithmetic); s up to the order of
    the prior's six-term sum."""
    from paper_2407_11349_amd.mcmc.hmc import leapfrog

    net = SurrogateNet(init_params(3))
    std = _std()
    sur = Surrogate(net, std)
    prior_var = 100.0

    def sur_post(z):
        ll, g = sur.value_and_grad(z)
        return float(ll[0]) - 0.5 * float(np.dot(z, z)) / prior_var, g[0] - np.asarray(z) / prior_var

    rng = np.random.default_rng(7)
    for trial in range(4):
        z0 = std.m_z + std.s_z * rng.normal(size=6)
        s0, g0 = sur_post(z0)
        p0 = rng.normal(size=6)
        inv_mass = std.s_z ** 2 * rng.uniform(0.5, 2.0, 6)
        eps, n = 0.05 * (trial + 1), [1, 7, 20, 20][trial]
        zh, ph, sh, gh = leapfrog(z0, p0, g0, eps, inv_mass, n, sur_post)
        zf, pf, sf, gf = sur.leapfrog(z0, p0, g0, eps, inv_mass, n, prior_var)
        assert np.array_equal(zf, zh) and np.array_equal(pf, ph) and np.array_equal(gf, gh), trial
        assert sf == pytest.approx(sh, rel=1e-15, abs=0.0)


def test_fused_leapfrog_stops_at_a_non_finite_step():
    net = SurrogateNet(init_params(3))
    std = _std()
    sur = Surrogate(net, std)
    z0 = std.m_z.copy()
    ll, g = sur.value_and_grad(z0)
    g0 = g[0] - z0 / 100.0
    p0 = np.ones(6)
    zf, pf, sf, gf = sur.leapfrog(z0, p0, g0, 1e200, np.ones(6), 5, 100.0)
    assert sf == -np.inf
    assert not np.all(np.isfinite(gf)) or not np.all(np.isfinite(zf))
    # the momentum after the first half step only (no step completed)
    np.testing.assert_array_equal(pf, p0 + (0.5 * 1e200) * g0)
