"""FP64 oracle of the network field and its losses (Sec. 2.D). TEST INFRASTRUCTURE ONLY:
imported by the test suite, the smoke check and the benchmark's CPU-baseline leg, never
by the GPU library; it shares no code with it.

The paper represents (T, p, u) by an MLP of the position, ties the BOS loss to it
through eta = 1 + rho0 G T0 / T, and adds a boundary loss and the Boussinesq residual
loss at collocation points (Sec. 2.D, Eq. (3)). It gives no architecture; the readings
taken here:

  * input: the position normalised to the field box, xhat = 2 (x - lo) / (hi - lo) - 1;
  * `depth` hidden layers of `width` units with tanh, then a linear layer to 5 outputs
    (T_nd, p, u_x, u_y, u_z), all nondimensional; T = T0 + (T_in - T0) T_nd, the
    paper's T_nd = (T - T0) / (T_in - T0) solved for T;
  * parameters packed as, per layer in order, the weight matrix [in][out] row-major then
    the bias [out] (3 -> width, width -> width (depth - 1 times), width -> 5);
  * the PDE is written in nondimensional coordinates x_nd = x / L, so a derivative in
    x_nd is L * 2 / (hi - lo) times the derivative in xhat on that axis; gravity e_g
    points along -z.

Forward values use NumPy (matmul, tanh). Derivatives with respect to the position and
the parameters are taken by PyTorch's automatic differentiation in float64 on the CPU
(a library primitive used as one step of the definition).
"""

from __future__ import annotations

from typing import Callable, Dict, Sequence, Tuple

import numpy as np
import torch

N_OUT = 5
E_G = (0.0, 0.0, -1.0)


def param_count(width: int, depth: int) -> int:
    return 3 * width + width + (depth - 1) * (width * width + width) + width * N_OUT + N_OUT


def layer_shapes(width: int, depth: int):
    dims = [3] + [width] * depth + [N_OUT]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def unpack(theta, width: int, depth: int):
    """[(W [in][out], b [out])] views of a packed parameter vector (NumPy or torch)."""
    out, o = [], 0
    for fi, fo in layer_shapes(width, depth):
        W = theta[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = theta[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == param_count(width, depth)
    return out


def normalise(x, lo, hi):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return 2.0 * (x - lo) / (hi - lo) - 1.0


def forward(theta: np.ndarray, width: int, depth: int, x: np.ndarray, lo, hi) -> np.ndarray:
    """MLP outputs [n][5] at positions x [n][3] (metres)."""
    a = normalise(np.asarray(x, np.float64), lo, hi)
    layers = unpack(np.asarray(theta, np.float64), width, depth)
    for W, b in layers[:-1]:
        a = np.tanh(a @ W + b)
    W, b = layers[-1]
    return a @ W + b


def temperature(out0: np.ndarray, T0: float, T_in: float) -> np.ndarray:
    return T0 + (T_in - T0) * out0


def voxel_centres(lo, hi, dims) -> np.ndarray:
    """Voxel-centre positions [nz * ny * nx][3], x fastest (the field's order)."""
    nx, ny, nz = dims
    ax = [lo[a] + (np.arange(n) + 0.5) * (hi[a] - lo[a]) / n for a, n in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


# ------------------------------------------------------------------------------------
# reverse mode with respect to the parameters
# ------------------------------------------------------------------------------------
def _torch_mlp(theta_t, width, depth, xhat_t):
    a = xhat_t
    layers = unpack(theta_t, width, depth)
    for W, b in layers[:-1]:
        a = torch.tanh(a @ W + b)
    W, b = layers[-1]
    return a @ W + b


def vjp_params(theta: np.ndarray, width: int, depth: int, x: np.ndarray, lo, hi, dL_dout: np.ndarray) -> np.ndarray:
    """sum_i dL/dout_i . d out_i / d theta (the parameter gradient of any loss whose
    derivative with respect to the outputs at the points x is dL_dout [n][5])."""
    th = torch.tensor(np.asarray(theta, np.float64), requires_grad=True)
    xh = torch.tensor(normalise(np.asarray(x, np.float64), lo, hi))
    out = _torch_mlp(th, width, depth, xh)
    out.backward(torch.tensor(np.asarray(dL_dout, np.float64)))
    return th.grad.numpy().copy()


def bos_temperature_seed(grad_delta: np.ndarray, T: np.ndarray, rho0G: float, T0: float, T_in: float) -> np.ndarray:
    """dL/dT_nd at the voxel centres from dL/d(eta - 1): eta - 1 = rho0G T0 / T gives
    d(eta - 1)/dT = -rho0G T0 / T^2, and dT/dT_nd = T_in - T0 (Sec. 2.A, 2.D)."""
    T = np.asarray(T, np.float64)
    return np.asarray(grad_delta, np.float64) * (-rho0G * T0 / (T * T)) * (T_in - T0)


def boundary_loss(theta, width, depth, x, lo, hi, target: np.ndarray, norms: Sequence[float]):
    """L_Gamma = sum_points sum_k ((target_k - out_k) / norm_k)^2 over the 5 outputs, each
    field divided by its normaliser (the paper's 'divided by its maximum value': the
    maximum |value| of that field's boundary data, one for the three velocity
    components). Returns (L, dL/dtheta)."""
    out = forward(theta, width, depth, x, lo, hi)
    nrm = np.asarray(norms, np.float64)
    r = (out - np.asarray(target, np.float64)) / nrm
    L = float(np.sum(r * r))
    return L, vjp_params(theta, width, depth, x, lo, hi, 2.0 * r / nrm)


def boundary_norms(target: np.ndarray) -> np.ndarray:
    t = np.asarray(target, np.float64)
    u = np.max(np.linalg.norm(t[:, 2:5], axis=1))
    return np.array([np.max(np.abs(t[:, 0])), np.max(np.abs(t[:, 1])), u, u, u])


# ------------------------------------------------------------------------------------
# Boussinesq residuals (Sec. 2.D) in nondimensional coordinates
# ------------------------------------------------------------------------------------
def jets(fields: Callable, x_nd: torch.Tensor):
    """Values [n][5], gradients [n][5][3] and second derivatives along each axis
    [n][5][3] of a field function x_nd -> (T_nd, p, u_x, u_y, u_z), by automatic
    differentiation (graph kept for a later backward pass)."""
    x_nd = x_nd.detach().requires_grad_(True)
    f = fields(x_nd)
    grads, seconds = [], []
    for k in range(N_OUT):
        g = torch.autograd.grad(f[:, k].sum(), x_nd, create_graph=True)[0]
        s = torch.stack([torch.autograd.grad(g[:, a].sum(), x_nd, create_graph=True)[0][:, a] for a in range(3)],
                        dim=1)
        grads.append(g)
        seconds.append(s)
    return f, torch.stack(grads, dim=1), torch.stack(seconds, dim=1)


def residuals(fields: Callable, x_nd: torch.Tensor, Re: float, Pe: float, Ri: float):
    """r_mass = div u; r_mom = (u . grad) u + grad p - lap(u) / Re + Ri T_nd e_g;
    r_heat = (u . grad) T_nd - lap(T_nd) / Pe (Sec. 2.D)."""
    f, g, s = jets(fields, x_nd)
    T, u = f[:, 0], f[:, 2:5]
    gT, gp, gu = g[:, 0], g[:, 1], g[:, 2:5]          # gu[i][k][a] = d u_k / d x_a
    lapT, lapu = s[:, 0].sum(1), s[:, 2:5].sum(2)
    r_mass = gu[:, 0, 0] + gu[:, 1, 1] + gu[:, 2, 2]
    conv = torch.einsum("ia,ika->ik", u, gu)           # (u . grad) u_k
    eg = torch.tensor(E_G, dtype=x_nd.dtype)
    r_mom = conv + gp - lapu / Re + Ri * T[:, None] * eg[None, :]
    r_heat = (u * gT).sum(1) - lapT / Pe
    return r_mass, r_mom, r_heat


def mlp_fields(theta_t: torch.Tensor, width: int, depth: int, lo, hi, L_ref: float) -> Callable:
    """x_nd -> MLP outputs, with xhat = 2 (L x_nd - lo) / (hi - lo) - 1."""
    lo_t = torch.tensor(np.asarray(lo, np.float64))
    hi_t = torch.tensor(np.asarray(hi, np.float64))

    def fields(x_nd):
        return _torch_mlp(theta_t, width, depth, 2.0 * (L_ref * x_nd - lo_t) / (hi_t - lo_t) - 1.0)

    return fields


def pde_loss(theta, width, depth, x, lo, hi, consts: Dict[str, float]) -> Tuple[float, np.ndarray]:
    """L_PDE = sum_i g1 r_mass^2 + g2 |r_mom|^2 + g3 r_heat^2 at the collocation points x
    [n][3] (metres); consts: Re, Pe, Ri, L (metres), g1, g2, g3. Returns (L, dL/dtheta)."""
    th = torch.tensor(np.asarray(theta, np.float64), requires_grad=True)
    x_nd = torch.tensor(np.asarray(x, np.float64) / consts["L"])
    rm, rv, rh = residuals(mlp_fields(th, width, depth, lo, hi, consts["L"]), x_nd, consts["Re"], consts["Pe"],
                           consts["Ri"])
    L = (consts["g1"] * (rm * rm).sum() + consts["g2"] * (rv * rv).sum() + consts["g3"] * (rh * rh).sum())
    (dth,) = torch.autograd.grad(L, th)
    return float(L.detach()), dth.numpy().copy()


def pde_residuals(theta, width, depth, x, lo, hi, consts):
    th = torch.tensor(np.asarray(theta, np.float64))
    x_nd = torch.tensor(np.asarray(x, np.float64) / consts["L"])
    rm, rv, rh = residuals(mlp_fields(th, width, depth, lo, hi, consts["L"]), x_nd, consts["Re"], consts["Pe"],
                           consts["Ri"])
    return rm.detach().numpy(), rv.detach().numpy(), rh.detach().numpy()
