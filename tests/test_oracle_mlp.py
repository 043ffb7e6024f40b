"""Pins for the oracle's network field and its losses (Sec. 2.D):

  * the forward pass against torch.nn's Linear/Tanh layers loaded with the same packed
    parameters (an independent implementation of the layers);
  * the parameter vector-Jacobian product against central differences;
  * position derivatives (gradient, second derivatives per axis) against central
    differences of the forward pass;
  * the Boussinesq residuals against exact solutions: Kovasznay's steady Navier-Stokes
    flow (momentum and mass residuals vanish), a stratified fluid at rest in hydrostatic
    balance (all residuals vanish: fixes the sign and direction of the buoyancy term),
    and steady 1D advection-diffusion T = exp(Pe x) (heat residual vanishes);
  * the PDE and boundary loss gradients against central differences in random
    parameter directions;
  * the BOS chain d(eta - 1)/dT_nd against central differences of the oracle's own
    eta(T), and the parameter gradient of a voxel-grid loss as the chain of the voxel
    gradient and central differences of the field in the parameters.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from bos_inputs import mlp_params
from oracle import mlp

W, D = 16, 3
LO, HI = (0.0, 0.0, 0.0), (4.0, 4.0, 3.0)
CONSTS = dict(Re=50.0, Pe=35.0, Ri=0.8, L=1.0, g1=1.0, g2=0.5, g3=2.0)


def _theta(seed=1, scale=1.0):
    return mlp_params(W, D, seed, out_scale=scale)


def _points(n, seed=2):
    rng = np.random.default_rng(seed)
    return rng.uniform(LO, HI, (n, 3))


def test_forward_matches_torch_nn_layers():
    th = _theta()
    th[np.arange(th.size) % 7 == 3] += 0.05  # non-zero biases too
    layers = []
    for (fi, fo), (Wm, b) in zip(mlp.layer_shapes(W, D), mlp.unpack(th, W, D)):
        lin = torch.nn.Linear(fi, fo).double()
        with torch.no_grad():
            lin.weight.copy_(torch.tensor(Wm.T))
            lin.bias.copy_(torch.tensor(b))
        layers += [lin, torch.nn.Tanh()]
    net = torch.nn.Sequential(*layers[:-1])
    x = _points(300)
    ref = net(torch.tensor(2.0 * (x - np.array(LO)) / (np.array(HI) - np.array(LO)) - 1.0)).detach().numpy()
    assert np.allclose(mlp.forward(th, W, D, x, LO, HI), ref, rtol=0, atol=1e-14)
    assert mlp.param_count(W, D) == th.size == 3 * 16 + 16 + 2 * (256 + 16) + 16 * 5 + 5


def test_param_vjp_matches_central_differences():
    th = _theta(3)
    x = _points(50)
    rng = np.random.default_rng(4)
    lam = rng.standard_normal((50, 5))
    g = mlp.vjp_params(th, W, D, x, LO, HI, lam)
    h = 1e-6
    for j in rng.choice(th.size, 25, replace=False):
        e = np.zeros_like(th)
        e[j] = h
        fd = (np.sum(lam * mlp.forward(th + e, W, D, x, LO, HI)) - np.sum(lam * mlp.forward(th - e, W, D, x, LO, HI))) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-7, abs=1e-9)


def test_position_derivatives_match_central_differences():
    th = _theta(5)
    x = _points(40)
    fields = mlp.mlp_fields(torch.tensor(th), W, D, LO, HI, 1.0)
    f, gr, s = mlp.jets(fields, torch.tensor(x))
    gr, s = gr.detach().numpy(), s.detach().numpy()
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1e-4
        fp, fm, f0 = (mlp.forward(th, W, D, x + sgn * e, LO, HI) for sgn in (1, -1, 0))
        assert np.allclose(gr[:, :, a], (fp - fm) / 2e-4, rtol=1e-6, atol=1e-8)
        assert np.allclose(s[:, :, a], (fp - 2 * f0 + fm) / 1e-8, rtol=1e-4, atol=1e-5)


def _kovasznay(Re):
    lam = Re / 2.0 - math.sqrt(Re * Re / 4.0 + 4.0 * math.pi ** 2)

    def fields(x):
        ex = torch.exp(lam * x[:, 0])
        u = 1.0 - ex * torch.cos(2 * math.pi * x[:, 1])
        v = lam / (2 * math.pi) * ex * torch.sin(2 * math.pi * x[:, 1])
        p = 0.5 * (1.0 - torch.exp(2 * lam * x[:, 0]))
        z = torch.zeros_like(u)
        return torch.stack([z, p, u, v, z], dim=1)

    return fields


def test_residuals_vanish_for_kovasznay_flow():
    x = torch.tensor(np.random.default_rng(6).uniform(-0.5, 1.0, (200, 3)))
    rm, rv, rh = mlp.residuals(_kovasznay(40.0), x, Re=40.0, Pe=10.0, Ri=3.0)
    assert rm.abs().max() < 1e-12 and rv.abs().max() < 1e-11 and rh.abs().max() < 1e-12
    # the same flow with the wrong Reynolds number leaves the viscous term unbalanced
    _, rv2, _ = mlp.residuals(_kovasznay(40.0), x, Re=20.0, Pe=10.0, Ri=3.0)
    assert rv2.abs().max() > 1e-2


def test_residuals_vanish_for_hydrostatic_stratified_rest():
    a, b, Ri = 0.3, -0.7, 2.5

    def fields(x):
        z = x[:, 2]
        T = a + b * z
        p = Ri * (a * z + 0.5 * b * z * z)  # dp/dz = Ri T: pressure gradient balances buoyancy
        zero = torch.zeros_like(z)
        return torch.stack([T, p, zero, zero, zero], dim=1)

    x = torch.tensor(np.random.default_rng(7).uniform(-1.0, 1.0, (100, 3)))
    rm, rv, rh = mlp.residuals(fields, x, Re=100.0, Pe=70.0, Ri=Ri)
    assert rm.abs().max() == 0 and rh.abs().max() < 1e-15 and rv.abs().max() < 1e-14
    # gravity reversed would need the opposite pressure gradient
    _, rv2, _ = mlp.residuals(fields, x, Re=100.0, Pe=70.0, Ri=-Ri)
    assert rv2[:, 2].abs().max() > 0.1


def test_heat_residual_vanishes_for_steady_advection_diffusion():
    Pe = 3.0

    def fields(x):
        one, zero = torch.ones_like(x[:, 0]), torch.zeros_like(x[:, 0])
        return torch.stack([torch.exp(Pe * x[:, 0]), zero, one, zero, zero], dim=1)

    x = torch.tensor(np.random.default_rng(8).uniform(-1.0, 1.0, (100, 3)))
    rm, _, rh = mlp.residuals(fields, x, Re=100.0, Pe=Pe, Ri=1.0)
    assert rm.abs().max() == 0 and rh.abs().max() < 1e-12


@pytest.mark.parametrize("loss", ["pde", "boundary"])
def test_loss_gradients_match_central_differences(loss):
    th = _theta(9, scale=0.5)
    x = _points(60, 10)
    if loss == "pde":
        def f(t):
            return mlp.pde_loss(t, W, D, x, LO, HI, CONSTS)
    else:
        tgt = mlp.forward(_theta(11), W, D, x, LO, HI)
        nrm = mlp.boundary_norms(tgt)

        def f(t):
            return mlp.boundary_loss(t, W, D, x, LO, HI, tgt, nrm)
    L, g = f(th)
    assert L > 0
    rng = np.random.default_rng(12)
    h = 1e-6
    for _ in range(6):
        d = rng.standard_normal(th.size)
        fd = (f(th + h * d)[0] - f(th - h * d)[0]) / (2 * h)
        assert fd == pytest.approx(float(g @ d), rel=1e-6)


def test_bos_temperature_chain():
    rng = np.random.default_rng(13)
    T = rng.uniform(288.0, 310.0, 50).astype(np.float32).astype(np.float64)
    gd = rng.standard_normal(50)
    T0, T_in, rho0G = 293.0, 303.0, 2.7e-4
    seed = mlp.bos_temperature_seed(gd, T, rho0G, T0, T_in)
    h = 1e-3
    dp = oracle.delta_from_temperature((T + h).astype(np.float32), rho0G, T0)
    dm = oracle.delta_from_temperature((T - h).astype(np.float32), rho0G, T0)
    # T +- h rounded to binary32 (spacing 3e-5 at 300 K): use the rounded step
    step = (T + h).astype(np.float32).astype(np.float64) - (T - h).astype(np.float32).astype(np.float64)
    fd = gd * (dp - dm) / step * (T_in - T0)
    assert np.allclose(seed, fd, rtol=1e-6)


def test_grid_parameter_gradient_is_the_chain_of_voxel_gradient_and_field_derivative():
    dims = (6, 5, 4)
    xc = mlp.voxel_centres(LO, HI, dims)
    assert xc.shape == (120, 3)
    assert np.allclose(xc[1] - xc[0], [4.0 / 6, 0, 0]) and np.allclose(xc[6] - xc[0], [0, 4.0 / 5, 0])
    th = _theta(14, scale=0.3)
    T0, T_in, rho0G = 293.0, 303.0, 2.7e-4
    rng = np.random.default_rng(15)
    g_delta = rng.standard_normal(120)

    def delta(t):
        T = mlp.temperature(mlp.forward(t, W, D, xc, LO, HI)[:, 0], T0, T_in)
        return rho0G * T0 / T

    T = mlp.temperature(mlp.forward(th, W, D, xc, LO, HI)[:, 0], T0, T_in)
    seed = np.zeros((120, 5))
    seed[:, 0] = mlp.bos_temperature_seed(g_delta, T, rho0G, T0, T_in)
    g = mlp.vjp_params(th, W, D, xc, LO, HI, seed)
    h = 1e-6
    for j in rng.choice(th.size, 20, replace=False):
        e = np.zeros_like(th)
        e[j] = h
        fd = g_delta @ (delta(th + e) - delta(th - e)) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-12)
