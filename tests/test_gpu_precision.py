"""GPU parity with 16-bit storage of eta - 1 (FP16 / BF16 codes q, eta - 1 = c + q / s with
s a power of two and c an offset), integrated in FP32.

Each case is compared with the oracle twice:
  * on the dequantised field (exactly the stored values): the arithmetic alone, held to
    the FP32 tolerances (exit point <= 1e-6 m, gradient rel-L2 < 1e-3);
  * on the unquantised field: storage + arithmetic, held to 1e-5 m at the exit point.

The storage default is the ambient offset c = rho0G (eta - 1 at T0 = 293 K): the codes hold
only the plume perturbation (|eta - 1 - c| <= 1.4e-5, s = 2^30) and the exit point stays
within 1e-5 m (measured at 256 x 256 rays: FP16 1.7e-7 m, BF16 1.2e-6 m).

Storage without an offset (c = 0, s = 2^25) does NOT meet the 1e-5 m bound and is kept only
as a labelled non-compliant comparison: the half-ulp of eta is 1.2e-7 (FP16) or 9.5e-7
(BF16); this rounding noise is independent per voxel, its gradient adds a random walk to
the deflection, and the exit error (FP16 2.7e-5 m = 2.7x the bound, BF16 1.7e-4 m = 17x,
roughly proportional to the half-ulp) exceeds even the RMS BOS displacement (2.1e-5 m).
Those cases assert that they miss the bound (so the claim stays true) and stay below a
regression ceiling.
"""

import numpy as np
import pytest
import torch

import oracle
from _common import RHO0G, exit_error, expected_scale, oracle_forward, room_workload, stored_delta
from paper_2509_14442_amd import api
from test_gpu_forward import DEV, _np, gpu_trace

pytestmark = pytest.mark.gpu

AMBIENT = RHO0G  # eta - 1 at the ambient temperature
EXIT_BOUND = 1e-5  # m, 16-bit storage against the exact field
COMPLIANT = [pytest.param("f16", AMBIENT, id="f16-ambient"), pytest.param("bf16", AMBIENT, id="bf16-ambient")]
# c = 0: (regression ceiling, measured miss factor over EXIT_BOUND)
NONCOMPLIANT = {"f16": (1e-4, 2.7), "bf16": (5e-4, 17.0)}
CASES = COMPLIANT + [pytest.param(d, 0.0, id=f"{d}-c0-noncompliant") for d in NONCOMPLIANT]


def _exact_delta(T32):
    return oracle.delta_from_temperature(T32.astype(np.float64), RHO0G)


def _forward_errors(dtype, offset):
    w = room_workload((128, 128, 128), 256, 256, seed=2)
    tr = gpu_trace(w, dtype, None, offset)
    scale = expected_scale(w.T32, dtype, offset)
    assert tr.scenes[0].field.scale == scale
    uv, ns = _np(tr.uv[0]), _np(tr.n_steps[0])
    fin = np.isfinite(uv[:, 0])

    _, ref = oracle_forward(w, stored_delta(w.T32, dtype, scale, offset))
    assert np.array_equal(fin, np.isfinite(ref["uv"][:, 0]))
    assert (ns != ref["n_steps"]).sum() <= 3
    e_arith = exit_error(uv[fin], ref["uv"][fin])
    assert e_arith.max() <= 1e-6, e_arith.max()

    _, ex = oracle_forward(w, _exact_delta(w.T32))
    ok = fin & np.isfinite(ex["uv"][:, 0])
    e_store = exit_error(uv[ok], ex["uv"][ok])
    disp = np.sqrt((ex["duv"][ok] ** 2).sum(1))
    print(f"{dtype} c={offset:g} s={scale:g}: exit vs dequantised max {e_arith.max():.2e} m, "
          f"vs exact max {e_store.max():.2e} m p99 {np.percentile(e_store, 99):.2e} m "
          f"({e_store.max() / EXIT_BOUND:.2f}x the {EXIT_BOUND:g} m bound), "
          f"BOS displacement rms {np.sqrt((disp ** 2).mean()):.2e} m")
    return e_store.max()


@pytest.mark.parametrize("dtype,offset", COMPLIANT)
def test_16bit_default_storage_meets_bound(dtype, offset):
    # the binding's default offset for 16-bit storage is the ambient one
    f = api.Field.from_temperature(torch.full((4, 4, 4), 300.0, device=DEV), dtype)
    assert f.offset == offset
    assert _forward_errors(dtype, offset) <= EXIT_BOUND


@pytest.mark.parametrize("dtype", list(NONCOMPLIANT), ids=[f"{d}-c0-noncompliant" for d in NONCOMPLIANT])
def test_16bit_without_offset_misses_bound(dtype):
    """Non-compliant comparison: c = 0 storage misses the 1e-5 m bound (by the factor in
    NONCOMPLIANT, measured); it is selectable but never the default."""
    ceiling, factor = NONCOMPLIANT[dtype]
    e = _forward_errors(dtype, 0.0)
    assert EXIT_BOUND < e <= ceiling, (e, factor)


@pytest.mark.parametrize("ckpt", [16, 4])
@pytest.mark.parametrize("dtype,offset", CASES)
def test_16bit_adjoint_against_dequantised(dtype, offset, ckpt):
    w = room_workload((64, 64, 48), 256, 256, seed=3, ckpt=ckpt)
    rng = np.random.default_rng(15)
    ids = np.sort(rng.choice(256 * 256, 4096, replace=False)).astype(np.int32)
    lam = rng.standard_normal((4096, 2)).astype(np.float32)
    field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), dtype, None, offset)
    sc = api.Scene(w.scene, field, torch.from_numpy(w.pattern32).to(DEV), torch.from_numpy(ids).to(DEV))
    tr = api.Tracer([sc])
    tr.forward()
    g = _np(tr.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0])
    scale = expected_scale(w.T32, dtype, offset)
    assert field.scale == scale
    F = oracle.grid_field(stored_delta(w.T32, dtype, scale, offset), w.scene.box_lo, w.scene.box_hi)
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64), ids)
    l2 = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert l2 < 1e-3, l2
