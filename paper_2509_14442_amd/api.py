"""Python binding of librbos: marshals torch device tensors into the C ABI.

PyTorch provides device memory and the stream; every step of the path runs in the
library's HIP kernels. There is no fallback: without librbos.so these functions raise.
"""

from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import torch

from . import _lib as L

# storage formats: code type, then "-xpair" for the x-pair layout (cell records otherwise)
DTYPES = {"f32": L.RBOS_F32, "f16": L.RBOS_F16, "bf16": L.RBOS_BF16,
          "f32-xpair": L.RBOS_F32_XPAIR, "f16-xpair": L.RBOS_F16_XPAIR, "bf16-xpair": L.RBOS_BF16_XPAIR}


def code_type(dtype: str) -> str:
    """"f32", "f16" or "bf16": the type of the stored codes."""
    return dtype.split("-")[0]
RHO0G = 2.7e-4  # rho0 * G of air at the ambient state used by the synthetic workloads
T_AMBIENT = 293.0


def lib():
    return L.load()


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return C.c_void_p(t.data_ptr())


class Field:
    """A packed eta - 1 field on the GPU (cell records of the corner codes)."""

    def __init__(self, dims: Sequence[int], dtype: str = "f32", scale: float = 1.0, offset: float = 0.0,
                 device="cuda"):
        nx, ny, nz = (int(d) for d in dims)
        self.dims = (nx, ny, nz)
        self.dtype = dtype
        self.code = DTYPES[dtype]
        self.scale = float(scale)
        self.offset = float(offset)
        nbytes = lib().rbos_field_bytes(nx, ny, nz, self.code)
        if nbytes == 0:
            raise ValueError(f"unsupported field shape {dims} / dtype {dtype}")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)

    @classmethod
    def from_temperature(cls, T: torch.Tensor, dtype: str = "f32", scale: Optional[float] = None,
                         offset: Optional[float] = None, rho0G: float = RHO0G, T0: float = T_AMBIENT, stream=None):
        """eta - 1 = rho0G * T0 / T from a [nz][ny][nx] float32 temperature tensor (kelvin).
        offset (None): the ambient eta - 1, rho0G, for 16-bit storage (the codes then hold
        only the perturbation), 0 for FP32. scale (None): the library's choice for the
        tensor's temperature range."""
        T = T.contiguous()
        if T.dtype != torch.float32 or T.dim() != 3:
            raise ValueError("T must be a float32 [nz][ny][nx] tensor")
        nz, ny, nx = T.shape
        if offset is None:
            offset = 0.0 if code_type(dtype) == "f32" else float(rho0G)
        if scale is None:
            tmin, tmax = (float(x) for x in torch.aminmax(T))
            scale = lib().rbos_code_scale_temperature(DTYPES[dtype], tmin, tmax, rho0G, T0, offset)
            if not scale > 0.0:
                raise ValueError(f"no code scale for temperatures in [{tmin}, {tmax}] K")
        f = cls((nx, ny, nz), dtype, scale, offset, T.device)
        f.rho0G, f.T0 = rho0G, T0
        f.encode_temperature(T, stream)
        return f

    def relayout(self, layout: str, stream=None) -> "Field":
        """A new field with the same codes in the other layout ("cell" or "xpair"), encoded
        from the source this field was last encoded from."""
        dtype = code_type(self.dtype) + ("-xpair" if layout == "xpair" else "")
        f = Field(self.dims, dtype, self.scale, self.offset, self.buf.device)
        if hasattr(self, "rho0G"):
            f.rho0G, f.T0 = self.rho0G, self.T0
            f.encode_temperature(self._keep, stream)
        else:
            f.encode(self._keep, stream)
        return f

    @property
    def layout(self) -> str:
        return "xpair" if self.dtype.endswith("-xpair") else "cell"

    def encode_temperature(self, T: torch.Tensor, stream=None):
        """Re-encode this field in place from a temperature tensor of the same shape."""
        T = T.contiguous()
        nx, ny, nz = self.dims
        if T.dtype != torch.float32 or tuple(T.shape) != (nz, ny, nx):
            raise ValueError("T must be a float32 [nz][ny][nx] tensor of this field's shape")
        L.check(lib().rbos_field_from_temperature(nx, ny, nz, _ptr(T), getattr(self, "rho0G", RHO0G),
                                                  getattr(self, "T0", T_AMBIENT), self.code, self.scale,
                                                  self.offset, _ptr(self.buf), _stream(stream)))
        self._keep = T

    @classmethod
    def from_delta(cls, delta: torch.Tensor, dtype: str = "f32", scale: Optional[float] = None,
                   offset: Optional[float] = None, stream=None):
        """Encode a given eta - 1 field ([nz][ny][nx] float32). offset (None): the middle of
        the field's range for 16-bit storage, 0 for FP32; scale (None): the library's choice
        for that range."""
        dmin, dmax = (float(x) for x in torch.aminmax(delta))
        if offset is None:
            offset = 0.0 if code_type(dtype) == "f32" else 0.5 * (dmin + dmax)
        if scale is None:
            scale = lib().rbos_code_scale(DTYPES[dtype], dmin, dmax, offset)
            if not scale > 0.0:
                raise ValueError(f"no code scale for eta - 1 in [{dmin}, {dmax}]")
        f = cls(tuple(reversed(delta.shape)), dtype, scale, offset, delta.device)
        f.encode(delta, stream)
        return f

    def encode(self, delta: torch.Tensor, stream=None):
        delta = delta.contiguous()
        if delta.dtype != torch.float32 or tuple(reversed(delta.shape)) != self.dims:
            raise ValueError("delta must be float32 with shape [nz][ny][nx] of this field")
        nx, ny, nz = self.dims
        L.check(lib().rbos_field_encode(nx, ny, nz, _ptr(delta), self.code, self.scale, self.offset,
                                        _ptr(self.buf), _stream(stream)))
        self._keep = delta


def _vec(x):
    return L.D3(*(float(v) for v in x))


class Scene:
    """One acquisition bound to device data. `desc` is any object with the geometry
    attributes of an rbos_scene (box_lo, cam_pos, wall_origin, step, ...)."""

    def __init__(self, desc, field: Field, pattern: Optional[torch.Tensor] = None,
                 pixel_ids: Optional[torch.Tensor] = None, ckpt_stride: Optional[int] = None):
        if tuple(field.dims) != tuple(desc.dims):
            raise ValueError(f"field dims {field.dims} != scene dims {desc.dims}")
        s = L.rbos_scene()
        s.nx, s.ny, s.nz = field.dims
        s.box_lo, s.box_hi = _vec(desc.box_lo), _vec(desc.box_hi)
        s.dtype, s.enc_scale, s.enc_offset = field.code, field.scale, field.offset
        s.field = field.buf.data_ptr()
        s.cam_pos, s.cam_fwd = _vec(desc.cam_pos), _vec(desc.cam_fwd)
        s.cam_right, s.cam_up = _vec(desc.cam_right), _vec(desc.cam_up)
        s.cam_fov_x_deg = desc.fov_x_deg
        s.width, s.height = desc.width, desc.height
        if pixel_ids is not None:
            pixel_ids = pixel_ids.to(device=field.buf.device, dtype=torch.int32).contiguous()
            s.pixel_ids = pixel_ids.data_ptr() if pixel_ids.numel() else field.buf.data_ptr()
            s.n_pixels = pixel_ids.numel()
        else:
            s.pixel_ids = None
            s.n_pixels = desc.width * desc.height
        s.wall_origin, s.wall_normal = _vec(desc.wall_origin), _vec(desc.wall_normal)
        s.wall_u, s.wall_v = _vec(desc.wall_u), _vec(desc.wall_v)
        s.wall_mode = desc.wall_mode
        if pattern is not None:
            pattern = pattern.to(device=field.buf.device, dtype=torch.float32).contiguous()
            if tuple(pattern.shape) != (desc.pat_h, desc.pat_w):
                raise ValueError("pattern shape must be (pat_h, pat_w)")
            s.pattern = pattern.data_ptr()
        s.pat_w, s.pat_h = desc.pat_w, desc.pat_h
        s.pat_extent_u, s.pat_extent_v = desc.pat_extent_u, desc.pat_extent_v
        s.proj_pos, s.proj_fwd = _vec(desc.proj_pos), _vec(desc.proj_fwd)
        s.proj_right, s.proj_up = _vec(desc.proj_right), _vec(desc.proj_up)
        s.proj_fov_x_deg = desc.proj_fov_x_deg
        s.step = desc.step
        s.max_steps = desc.max_steps
        s.ckpt_stride = desc.ckpt_stride if ckpt_stride is None else int(ckpt_stride)
        s.tracer = int(getattr(desc, "tracer", L.RBOS_TRACER_NONLINEAR))
        s.spp = int(getattr(desc, "spp", 1))
        s.seed = int(getattr(desc, "seed", 0))
        s.radiometry = int(getattr(desc, "radiometry", 0))
        self.struct = s
        self.desc = desc
        self.field = field
        self.pattern = pattern
        self.pixel_ids = pixel_ids
        self.n_pixels = int(s.n_pixels)
        self.spp = int(s.spp)
        self.n_rays = self.n_pixels * self.spp  # ray r = sample r // n_pixels of pixel r % n_pixels
        self.radiometry = bool(s.radiometry)
        self.dims = field.dims

    def set_field(self, field: Field):
        self.field = field
        self.struct.field = field.buf.data_ptr()
        self.struct.dtype, self.struct.enc_scale, self.struct.enc_offset = field.code, field.scale, field.offset


def make_launch(tile=(8, 8), waves_per_block=4, persistent=False, blocks_per_cu=0) -> L.rbos_launch:
    l = L.rbos_launch()
    l.tile_w, l.tile_h = tile
    l.waves_per_block = waves_per_block
    l.persistent = 1 if persistent else 0
    l.blocks_per_cu = blocks_per_cu
    return l


class Tracer:
    """Output buffers, workspace and the three ABI calls for a batch of scenes."""

    def __init__(self, scenes: List[Scene], launch: Optional[L.rbos_launch] = None, checkpoints: bool = True,
                 adjoint_launch: Optional[L.rbos_launch] = None, want_dir: bool = False):
        """`launch` shapes the forward trace and, unless `adjoint_launch` is given, the
        adjoint too (checkpoints are stored per ray, so the two may differ). Per-ray
        buffers hold n_pixels * spp rays, sample-major; images hold n_pixels values."""
        self.scenes = scenes
        self.n = len(scenes)
        self.launch = launch
        self.adjoint_launch = adjoint_launch if adjoint_launch is not None else launch
        self._arr = (L.rbos_scene * max(self.n, 1))(*[s.struct for s in scenes])
        dev = scenes[0].field.buf.device if scenes else torch.device("cuda")
        ws = lib().rbos_workspace_bytes(self._arr, self.n)
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
        self.uv, self.duv, self.n_steps, self.status, self.ckpt, self.wall_dir = [], [], [], [], [], []
        self._outs = (L.rbos_trace_out * max(self.n, 1))()
        for i, s in enumerate(scenes):
            n = s.n_rays
            self.uv.append(torch.empty((n, 2), dtype=torch.float32, device=dev))
            self.duv.append(torch.empty((n, 2), dtype=torch.float32, device=dev))
            self.n_steps.append(torch.empty(n, dtype=torch.int32, device=dev))
            self.status.append(torch.empty(n, dtype=torch.uint8, device=dev))
            # the wall direction: needed by the radiometric weight, kept when asked for
            wd = torch.empty((n, 3), dtype=torch.float32, device=dev) if (s.radiometry or want_dir) else None
            self.wall_dir.append(wd)
            cb = lib().rbos_ckpt_bytes(C.byref(self._arr[i])) if checkpoints else 0
            self.ckpt.append(torch.empty(max(cb // 4, 1), dtype=torch.float32, device=dev) if cb else None)
            o = self._outs[i]
            o.wall_uv, o.wall_duv = self.uv[i].data_ptr(), self.duv[i].data_ptr()
            o.n_steps, o.status = self.n_steps[i].data_ptr(), self.status[i].data_ptr()
            o.ckpt = self.ckpt[i].data_ptr() if self.ckpt[i] is not None else None
            o.wall_dir = wd.data_ptr() if wd is not None else None
        if not checkpoints:
            for i in range(self.n):
                self._arr[i].ckpt_stride = 0

    def refresh(self):
        """Re-read the scene structs (e.g. after Scene.set_field)."""
        for i, s in enumerate(self.scenes):
            stride = self._arr[i].ckpt_stride
            self._arr[i] = s.struct
            self._arr[i].ckpt_stride = stride

    def _launch_ptr(self):
        return C.byref(self.launch) if self.launch is not None else None

    def _adjoint_launch_ptr(self):
        return C.byref(self.adjoint_launch) if self.adjoint_launch is not None else None

    def forward(self, stream=None):
        L.check(lib().rbos_trace_forward(self._arr, self.n, self._outs, self._launch_ptr(),
                                         _ptr(self.workspace), self.workspace.numel(), _stream(stream)))
        return self

    def render(self, targets: Optional[List[Optional[torch.Tensor]]] = None, want_grad: bool = True, stream=None):
        """Images (and with targets: L_BOS and dL/d(u, v)). Output buffers are reused
        across calls with the same targets, so repeated calls allocate nothing."""
        dev = self.workspace.device
        key = (tuple(None if t is None else t.data_ptr() for t in targets) if targets is not None else None,
               want_grad)
        if getattr(self, "_render_key", None) != key:
            io = (L.rbos_render_io * max(self.n, 1))()
            self.image, self.dL_duv, self.dL_ddir, self.loss = [], [], [], []
            self._targets = []
            for i, s in enumerate(self.scenes):
                img = torch.empty(s.n_pixels, dtype=torch.float32, device=dev)
                tgt = targets[i] if targets is not None else None
                if tgt is not None:
                    tgt = tgt.to(device=dev, dtype=torch.float32).contiguous().reshape(-1)
                    if tgt.numel() != s.n_pixels:
                        raise ValueError(f"target has {tgt.numel()} values for {s.n_pixels} pixels")
                g = (torch.empty((s.n_rays, 2), dtype=torch.float32, device=dev)
                     if (tgt is not None and want_grad) else None)
                gd = (torch.empty((s.n_rays, 3), dtype=torch.float32, device=dev)
                      if (g is not None and s.radiometry) else None)
                lo = torch.zeros(1, dtype=torch.float32, device=dev) if tgt is not None else None
                io[i].target, io[i].image = _ptr(tgt), _ptr(img)
                io[i].dL_duv, io[i].loss, io[i].dL_ddir = _ptr(g), _ptr(lo), _ptr(gd)
                self.image.append(img)
                self.dL_duv.append(g)
                self.dL_ddir.append(gd)
                self.loss.append(lo)
                self._targets.append(tgt)
            self._render_io = io
            self._render_key = key
        L.check(lib().rbos_render(self._arr, self.n, self._outs, self._render_io, _ptr(self.workspace),
                                  self.workspace.numel(), _stream(stream)))
        return self

    def adjoint(self, grads: Optional[List[torch.Tensor]] = None, dL_duv: Optional[List[torch.Tensor]] = None,
                zero: bool = True, stream=None,
                dL_ddir: Optional[List[Optional[torch.Tensor]]] = None, noalloc: bool = False) -> List[torch.Tensor]:
        """dL/d(eta - 1) per scene (float64 [nz][ny][nx]); accumulates into `grads` if given.
        Without explicit per-ray seeds, uses the last render's dL/d(u, v) (and, with the
        radiometric weight, dL/d(direction)). noalloc: call rbos_trace_adjoint_noalloc, which
        keeps its scratch in the library's static device array instead of the workspace."""
        dev = self.workspace.device
        if dL_duv is None:
            dL = self.dL_duv
            if dL_ddir is None:
                dL_ddir = getattr(self, "dL_ddir", None)
        else:
            dL = dL_duv
        if grads is None:
            grads = [torch.zeros(tuple(reversed(s.dims)), dtype=torch.float64, device=dev) for s in self.scenes]
        elif zero:
            for g in grads:
                g.zero_()
        io = (L.rbos_adjoint_io * max(self.n, 1))()
        keep = []
        for i in range(self.n):
            d = dL[i].to(device=dev, dtype=torch.float32).contiguous()
            keep.append(d)
            io[i].dL_duv, io[i].grad = _ptr(d), _ptr(grads[i])
            dd = dL_ddir[i] if dL_ddir is not None else None
            if dd is not None:
                dd = dd.to(device=dev, dtype=torch.float32).contiguous()
                keep.append(dd)
            io[i].dL_ddir = _ptr(dd)
        if noalloc:
            L.check(lib().rbos_trace_adjoint_noalloc(self._arr, self.n, self._outs, io, self._adjoint_launch_ptr(),
                                                     _stream(stream)))
        else:
            L.check(lib().rbos_trace_adjoint(self._arr, self.n, self._outs, io, self._adjoint_launch_ptr(),
                                             _ptr(self.workspace), self.workspace.numel(), _stream(stream)))
        self._keep_adj = keep
        return grads


class MLP:
    """The network field of Sec. 2.D on the GPU: (T_nd, p, u) = MLP(xhat; params), tanh
    hidden layers, packed FP32 parameters (see include/rbos.h). Each point set (a points
    tensor or a voxel grid) keeps its own workspace, which holds the activations of its
    last forward for the backward."""

    def __init__(self, params: torch.Tensor, width: int, depth: int, box_lo, box_hi):
        n = lib().rbos_mlp_param_count(width, depth)
        if n == 0:
            raise ValueError(f"unsupported MLP width {width} / depth {depth}")
        if params.numel() != n or params.dtype != torch.float32 or not params.is_cuda:
            raise ValueError(f"params must be a float32 GPU tensor of {n} values")
        self.params = params.contiguous()
        self.width, self.depth = width, depth
        m = L.rbos_mlp()
        m.width, m.depth = width, depth
        m.params = self.params.data_ptr()
        m.box_lo, m.box_hi = _vec(box_lo), _vec(box_hi)
        self.struct = m
        self._ws = {}

    @staticmethod
    def param_count(width: int, depth: int) -> int:
        return int(lib().rbos_mlp_param_count(width, depth))

    def _set(self, points, grid):
        if points is not None:
            points = points.contiguous()
            if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
                raise ValueError("points must be float32 [n][3]")
            n, key, g = points.shape[0], ("p", points.data_ptr(), points.shape[0]), None
        else:
            nx, ny, nz = (int(v) for v in grid)
            n, key, g = nx * ny * nz, ("g", nx, ny, nz), (C.c_int32 * 3)(nx, ny, nz)
        if key not in self._ws:
            nb = lib().rbos_mlp_workspace_bytes(self.width, self.depth, n)
            self._ws[key] = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.params.device)
        return points, n, g, self._ws[key]

    def forward(self, points: Optional[torch.Tensor] = None, grid=None, want_out: bool = True,
                T0: Optional[float] = None, T_in: Optional[float] = None, stream=None):
        """Outputs [n][5] (if want_out) and, with T0 and T_in, T [n] = T0 + (T_in - T0) out_0."""
        points, n, g, ws = self._set(points, grid)
        dev = self.params.device
        out = torch.empty((n, 5), dtype=torch.float32, device=dev) if want_out else None
        T = torch.empty(n, dtype=torch.float32, device=dev) if T0 is not None else None
        L.check(lib().rbos_mlp_forward(C.byref(self.struct), _ptr(points), n, g, _ptr(out), _ptr(T),
                                       float(T0 or 0.0), float(T_in or 0.0), _ptr(ws), ws.numel(), _stream(stream)))
        self._keep = points
        return out, T

    def backward(self, dL_dout: torch.Tensor, points: Optional[torch.Tensor] = None, grid=None,
                 dparams: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """dparams += sum_i dL_dout_i . d out_i / d params (after forward on the same points)."""
        points, n, g, ws = self._set(points, grid)
        if dparams is None:
            dparams = torch.zeros_like(self.params)
        d = dL_dout.to(dtype=torch.float32).contiguous()
        if tuple(d.shape) != (n, 5):
            raise ValueError(f"dL_dout must be [{n}][5]")
        L.check(lib().rbos_mlp_backward(C.byref(self.struct), _ptr(points), n, g, _ptr(d), _ptr(dparams), _ptr(ws),
                                        ws.numel(), _stream(stream)))
        self._keep_d = d
        return dparams

    def pde_loss(self, points: torch.Tensor, Re: float, Pe: float, Ri: float, L_ref: float, gamma=(1.0, 1.0, 1.0),
                 dparams: Optional[torch.Tensor] = None, want_grad: bool = True, want_residuals: bool = False,
                 stream=None):
        """Boussinesq residual loss at collocation points [n][3]: (loss [1], dparams (added
        into if given), residuals [n][5] or None)."""
        points = points.contiguous()
        n = points.shape[0]
        dev = self.params.device
        key = ("pde", n)
        if key not in self._ws:
            nb = lib().rbos_mlp_pde_workspace_bytes(self.width, self.depth, n)
            self._ws[key] = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        ws = self._ws[key]
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        if want_grad and dparams is None:
            dparams = torch.zeros_like(self.params)
        res = torch.empty((n, 5), dtype=torch.float32, device=dev) if want_residuals else None
        pde = L.rbos_pde(Re, Pe, Ri, L_ref, L.D3(*gamma))
        L.check(lib().rbos_mlp_pde_loss(C.byref(self.struct), C.byref(pde), _ptr(points), n, _ptr(loss),
                                        _ptr(dparams) if want_grad else None, _ptr(res), _ptr(ws), ws.numel(),
                                        _stream(stream)))
        self._keep = points
        return loss, (dparams if want_grad else None), res

    @staticmethod
    def bos_seed(T: torch.Tensor, grad_delta: torch.Tensor, T0: float, T_in: float, rho0G: float = RHO0G,
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """dL/dout at the voxel centres from dL/d(eta - 1) (float64) and T (kelvin)."""
        n = T.numel()
        if out is None:
            out = torch.empty((n, 5), dtype=torch.float32, device=T.device)
        L.check(lib().rbos_mlp_bos_seed(n, _ptr(T.contiguous()), _ptr(grad_delta.contiguous()), rho0G, T0, T_in,
                                        _ptr(out), _stream(stream)))
        return out


def fit_seed(out: torch.Tensor, target: torch.Tensor, norms, want_loss: bool = True, stream=None):
    """Boundary loss sum ((out - target) / norm)^2 over [n][5] outputs: (seed dL/dout, loss)."""
    n = out.shape[0]
    o, t = out.contiguous(), target.to(dtype=torch.float32).contiguous()
    dL = torch.empty_like(o)
    loss = torch.zeros(1, dtype=torch.float32, device=o.device) if want_loss else None
    nb = lib().rbos_mlp_fit_workspace_bytes(n)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=o.device)
    nrm = (C.c_double * 5)(*(float(v) for v in norms))
    L.check(lib().rbos_mlp_fit_seed(n, _ptr(o), _ptr(t), nrm, _ptr(dL), _ptr(loss), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return dL, loss


class BOSLoss(torch.autograd.Function):
    """L_BOS(eta - 1) for one scene, with the hand-written adjoint as its backward.

    forward(delta [nz][ny][nx] float32, tracer, target [n_pixels]) -> scalar loss.
    The tracer's scene must use an FP32 field whose buffer this function re-encodes."""

    @staticmethod
    def forward(ctx, delta, tracer: Tracer, target):
        sc = tracer.scenes[0]
        sc.field.encode(delta.detach())
        tracer.forward().render([target])
        ctx.tracer = tracer
        ctx.shape = delta.shape
        return tracer.loss[0].reshape(()).clone()

    @staticmethod
    def backward(ctx, g):
        tr = ctx.tracer
        grads = tr.adjoint()
        return (grads[0] * g.to(torch.float64)).to(torch.float32), None, None


def bos_loss(delta: torch.Tensor, tracer: Tracer, target: torch.Tensor) -> torch.Tensor:
    return BOSLoss.apply(delta, tracer, target)
