"""GPU parity of the network field (Sec. 2.D) against the oracle: the MLP forward at
arbitrary points and at the voxel centres (FP32 on the matrix cores vs FP64; depths 1 to
the largest, 8), its
parameter gradient for given per-point output seeds, and the BOS loss's parameter
gradient end to end (MLP -> T on the voxel grid -> eta -> trace -> render -> adjoint ->
chain to T_nd -> MLP backward).

Tolerances: outputs are O(1) sums of 64 FP32 products per layer through tanh, so
|out - oracle| <= 2e-5 (measured ~1e-6); T = T0 + 10 K out_0 within 3e-4 K; parameter
gradients rel-L2 < 1e-5 for given seeds (FP32 accumulation over <= 2^17 points), and
< 1e-3 end to end, where the seeds themselves come from the FP32 tracer.
"""

import numpy as np
import pytest
import torch

import oracle
from bos_inputs import mlp_params
from oracle import mlp as omlp
from _common import grad_errors, stored_delta
from bos_inputs import binary_dots, scene_unit_box
from paper_2509_14442_amd import api
from test_gpu_forward import DEV, _np

pytestmark = pytest.mark.gpu

LO, HI = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
T0, T_IN = 293.0, 303.0


def _mlp(depth, seed=1, scale=1.0):
    th = mlp_params(64, depth, seed, out_scale=scale)
    th[np.arange(th.size) % 5 == 2] += 0.02  # non-zero biases
    m = api.MLP(torch.from_numpy(th.astype(np.float32)).to(DEV), 64, depth, LO, HI)
    return m, th.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("depth,n", [(1, 1), (3, 1000), (4, 4099), (6, 333), (8, 257)])
def test_forward_at_points(depth, n):
    m, th = _mlp(depth)
    x = np.random.default_rng(depth).uniform(LO, HI, (n, 3)).astype(np.float32)
    out, T = m.forward(torch.from_numpy(x).to(DEV), T0=T0, T_in=T_IN)
    ref = omlp.forward(th, 64, depth, x.astype(np.float64), LO, HI)
    err = np.abs(_np(out) - ref).max()
    print(f"depth {depth}, {n} points: max |out - oracle| {err:.2e}")
    assert err <= 2e-5
    assert np.abs(_np(T) - omlp.temperature(ref[:, 0], T0, T_IN)).max() <= 3e-4


def test_forward_on_the_voxel_grid():
    m, th = _mlp(4, 2)
    dims = (24, 20, 17)
    out, T = m.forward(grid=dims, T0=T0, T_in=T_IN)
    ref = omlp.forward(th, 64, 4, omlp.voxel_centres(LO, HI, dims), LO, HI)
    assert np.abs(_np(out) - ref).max() <= 2e-5
    assert np.abs(_np(T) - omlp.temperature(ref[:, 0], T0, T_IN)).max() <= 3e-4


@pytest.mark.parametrize("depth,n", [(1, 70), (4, 5000), (5, 131072), (8, 3001)])
def test_parameter_gradient_for_given_seeds(depth, n):
    m, th = _mlp(depth, 3)
    rng = np.random.default_rng(10 + depth)
    x = rng.uniform(LO, HI, (n, 3)).astype(np.float32)
    lam = rng.standard_normal((n, 5)).astype(np.float32)
    xt = torch.from_numpy(x).to(DEV)
    m.forward(xt, want_out=False)
    g = _np(m.backward(torch.from_numpy(lam).to(DEV), xt)).astype(np.float64)
    ref = omlp.vjp_params(th, 64, depth, x.astype(np.float64), LO, HI, lam.astype(np.float64))
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    print(f"depth {depth}, {n} points: dparams rel-L2 {rel:.2e}")
    assert rel < 1e-5
    assert np.abs(g - ref).max() <= 1e-4 * np.abs(ref).max()
    # accumulation: a second backward adds the same gradient again
    d2 = m.backward(torch.from_numpy(lam).to(DEV), xt, dparams=torch.from_numpy(g.astype(np.float32)).to(DEV))
    assert np.allclose(_np(d2), 2 * g, rtol=1e-6, atol=1e-6 * np.abs(g).max())


def test_backward_is_deterministic():
    m, _ = _mlp(4, 4)
    x = torch.from_numpy(np.random.default_rng(5).uniform(LO, HI, (70000, 3)).astype(np.float32)).to(DEV)
    lam = torch.from_numpy(np.random.default_rng(6).standard_normal((70000, 5)).astype(np.float32)).to(DEV)
    m.forward(x, want_out=False)
    g1 = m.backward(lam, x)
    g2 = m.backward(lam, x)
    assert torch.equal(g1, g2)


def test_bos_loss_parameter_gradient_end_to_end():
    """Unit-box scene on a 32^3 grid whose temperatures come from the MLP; target image
    from a second network."""
    sc = scene_unit_box().replace(width=48, height=48)
    dims = sc.dims
    m, th = _mlp(3, 7, scale=0.3)
    _, th2 = _mlp(3, 8, scale=0.3)
    pat = binary_dots(11)
    # target: the oracle's render of the second network's field
    xc = omlp.voxel_centres(LO, HI, dims)
    T2 = omlp.temperature(omlp.forward(th2, 64, 3, xc, LO, HI)[:, 0], T0, T_IN).reshape(dims[::-1])
    F2 = oracle.grid_field(stored_delta(T2.astype(np.float32)), LO, HI)
    fw2 = oracle.trace(F2, sc)
    target = oracle.render(sc, pat, fw2["uv"], fw2["status"])[0]

    # GPU: MLP -> T grid -> field -> trace -> render -> adjoint -> seed -> backward
    _, T = m.forward(grid=dims, want_out=False, T0=T0, T_in=T_IN)
    field = api.Field.from_temperature(T.reshape(dims[::-1]), "f32")
    scene = api.Scene(sc, field, torch.from_numpy(pat.astype(np.float32)).to(DEV))
    tr = api.Tracer([scene])
    tr.forward().render([torch.from_numpy(target.astype(np.float32)).to(DEV)])
    g_delta = tr.adjoint()[0].reshape(-1)
    seed = api.MLP.bos_seed(T, g_delta, T0, T_IN)
    g = _np(m.backward(seed, grid=dims)).astype(np.float64)

    # oracle: the same chain in FP64 from its own evaluation of the network (its
    # temperatures rounded to binary32, as the field is stored; they differ from the
    # GPU's by ~1e-5 K, i.e. ~1e-11 in eta - 1)
    T_or = omlp.temperature(omlp.forward(th, 64, 3, xc, LO, HI)[:, 0], T0, T_IN).reshape(dims[::-1])
    assert np.abs(_np(T).reshape(dims[::-1]) - T_or).max() <= 3e-4
    T32 = T_or.astype(np.float32)
    F = oracle.grid_field(stored_delta(T32), LO, HI)
    fw = oracle.trace(F, sc)
    img, dI, _ = oracle.render(sc, pat, fw["uv"], fw["status"])
    L, dL = oracle.loss(img, target, dI)
    assert float(tr.loss[0]) == pytest.approx(L, rel=1e-4)
    gd_ref = oracle.adjoint(F, sc, dL)
    s_ref = np.zeros((xc.shape[0], 5))
    s_ref[:, 0] = omlp.bos_temperature_seed(gd_ref.ravel(), T_or.ravel(), 2.7e-4, T0, T_IN)
    assert np.abs(_np(seed)[:, 0] - s_ref[:, 0]).max() <= 1e-3 * np.abs(s_ref[:, 0]).max()
    assert not _np(seed)[:, 1:].any()
    ref = omlp.vjp_params(th, 64, 3, xc, LO, HI, s_ref)
    l2, _ = grad_errors(g, ref)
    print(f"end-to-end dparams rel-L2 {l2:.2e}")
    assert l2 < 1e-3


def test_boundary_loss_and_gradient():
    """Boundary loss on the x = lo face (the paper's inlet plane), targets from a second
    network, normalisers from the targets."""
    m, th = _mlp(4, 20, scale=0.5)
    _, th_t = _mlp(4, 21, scale=0.5)
    rng = np.random.default_rng(22)
    n = 4096 + 17
    x = np.column_stack([np.full(n, LO[0]), rng.uniform(LO[1], HI[1], n), rng.uniform(LO[2], HI[2], n)])
    x = x.astype(np.float32)
    tgt = omlp.forward(th_t, 64, 4, x.astype(np.float64), LO, HI)
    norms = omlp.boundary_norms(tgt)
    L_ref, g_ref = omlp.boundary_loss(th, 64, 4, x.astype(np.float64), LO, HI, tgt, norms)
    xt = torch.from_numpy(x).to(DEV)
    out, _ = m.forward(xt)
    dL, loss = api.fit_seed(out, torch.from_numpy(tgt.astype(np.float32)).to(DEV), norms)
    g = _np(m.backward(dL, xt)).astype(np.float64)
    assert float(loss[0]) == pytest.approx(L_ref, rel=1e-5)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"boundary loss {float(loss[0]):.6g} (oracle {L_ref:.6g}), dparams rel-L2 {rel:.2e}")
    assert rel < 1e-5


PDE = dict(Re=50.0, Pe=35.0, Ri=0.8, L=0.5, g1=1.0, g2=0.5, g3=2.0)


@pytest.mark.parametrize("depth,n", [(1, 37), (3, 2000), (4, 8192), (8, 500)])
def test_pde_loss_residuals_and_gradient(depth, n):
    """The paper's mini-batch holds 8192 collocation points per step."""
    m, th = _mlp(depth, 30 + depth, scale=0.5)
    rng = np.random.default_rng(40 + depth)
    x = rng.uniform(LO, HI, (n, 3)).astype(np.float32)
    x64 = x.astype(np.float64)
    L_ref, g_ref = omlp.pde_loss(th, 64, depth, x64, LO, HI, PDE)
    rm, rv, rh = omlp.pde_residuals(th, 64, depth, x64, LO, HI, PDE)
    res_ref = np.column_stack([rm, rv, rh])
    loss, g, res = m.pde_loss(torch.from_numpy(x).to(DEV), PDE["Re"], PDE["Pe"], PDE["Ri"], PDE["L"],
                              (PDE["g1"], PDE["g2"], PDE["g3"]), want_residuals=True)
    res, g = _np(res).astype(np.float64), _np(g).astype(np.float64)
    e_res = np.abs(res - res_ref).max() / np.abs(res_ref).max()
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"depth {depth}, {n} points: loss {float(loss[0]):.6g} (oracle {L_ref:.6g}), residuals max err "
          f"{e_res:.2e} of max, dparams rel-L2 {rel:.2e}")
    assert float(loss[0]) == pytest.approx(L_ref, rel=1e-4)
    assert e_res < 1e-4
    assert rel < 1e-4
    # loss and residuals alone (no gradient) give the same values
    loss2, g2, _ = m.pde_loss(torch.from_numpy(x).to(DEV), PDE["Re"], PDE["Pe"], PDE["Ri"], PDE["L"],
                              (PDE["g1"], PDE["g2"], PDE["g3"]), want_grad=False)
    assert g2 is None and float(loss2[0]) == float(loss[0])


def test_network_field_at_bench_size():
    """The network field as the benchmark runs it: depth 4 on the 128^3 voxel centres of the
    4 x 4 x 3 m room (2,097,152 points, the largest launch of these kernels), checked on
    4096 sampled voxels: the outputs and T there, and the parameter gradient of seeds
    that are non-zero only at those voxels (so the oracle needs only them)."""
    import bos_inputs as bi

    lo, hi, dims = (0.0, 0.0, 0.0), (4.0, 4.0, 3.0), (128, 128, 128)
    th = bi.mlp_params(64, 4, 3, out_scale=0.3, bias_std=0.05).astype(np.float32)
    m = api.MLP(torch.from_numpy(th).to(DEV), 64, 4, lo, hi)
    th64 = th.astype(np.float64)
    out, T = m.forward(grid=dims, T0=T0, T_in=T_IN)
    n = 128 ** 3
    rng = np.random.default_rng(50)
    idx = np.sort(rng.choice(n, 4096, replace=False))
    xc = omlp.voxel_centres(lo, hi, dims)[idx]
    ref = omlp.forward(th64, 64, 4, xc, lo, hi)
    got = _np(out)[idx].astype(np.float64)
    assert np.abs(got - ref).max() <= 2e-5
    assert np.abs(_np(T)[idx] - omlp.temperature(ref[:, 0], T0, T_IN)).max() <= 3e-4
    lam = np.zeros((n, 5), np.float32)
    lam[idx] = rng.standard_normal((4096, 5)).astype(np.float32)
    g = _np(m.backward(torch.from_numpy(lam).to(DEV), grid=dims)).astype(np.float64)
    g_ref = omlp.vjp_params(th64, 64, 4, xc, lo, hi, lam[idx].astype(np.float64))
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"128^3 grid: max |out - oracle| {np.abs(got - ref).max():.2e} on 4096 voxels, dparams rel-L2 {rel:.2e}")
    assert rel < 1e-5
