"""Torch-tensor front end of the C ABI.

Each function checks tensor devices / dtypes, allocates outputs with torch
(the caching allocator supplies device memory) and calls the library on the
current HIP stream.  No computation of the method happens here.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check, load


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")


from .layout import blocks, latent_width, line_stride  # noqa: E402,F401


def to_blocked(z: torch.Tensor, k: int | None = None) -> torch.Tensor:
    """Re-pack plain (m, k) codes into the blocked RGBx layout (m, 4B)."""
    k = k or z.shape[1]
    m = z.shape[0]
    out = torch.zeros(m, blocks(k), 4, dtype=z.dtype, device=z.device)
    zp = torch.zeros(m, 3 * blocks(k), dtype=z.dtype, device=z.device)
    zp[:, :k] = z
    out[:, :, :3] = zp.view(m, blocks(k), 3)
    return out.view(m, latent_width(k))


def from_blocked(zb: torch.Tensor, k: int) -> torch.Tensor:
    """Plain (m, k) view of blocked RGBx rows."""
    m = zb.shape[0]
    return zb[:, :latent_width(k)].reshape(m, blocks(k), 4)[:, :, :3].reshape(m, 3 * blocks(k))[:, :k]


def padded(x: torch.Tensor, ld: int | None = None) -> torch.Tensor:
    """Copy of a (m, n) float32 tensor with rows padded to a multiple of 4 floats."""
    m, n = x.shape
    ld = ld or 4 * ((n + 3) // 4)
    out = torch.zeros(m, ld, dtype=torch.float32, device=x.device)
    out[:, :n] = x
    return out


@dataclass
class Paths:
    """Device light-path records (see include/hc.h for the format)."""
    hdr: torch.Tensor        # uint32 / int32 [n_pixels * spp]
    pix_first: torch.Tensor  # [n_pixels]
    vtx: torch.Tensor        # [n_vertices, 2]
    n_pixels: int
    spp: int

    @property
    def n_vertices(self) -> int:
        return int(self.vtx.shape[0]) if self.vtx is not None else 0

    def c(self) -> _lib.Paths:
        return _lib.Paths(self.n_pixels, self.spp, 0, self.hdr.data_ptr(), self.pix_first.data_ptr(),
                          self.vtx.data_ptr() if self.n_vertices else None, self.n_vertices)

    @staticmethod
    def from_numpy(hdr, pix_first, vtx, spp: int, device="cuda") -> "Paths":
        import numpy as np
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(device)  # noqa: E731
        vt = t(vtx.reshape(-1, 2)) if vtx.size else torch.zeros(0, 2, dtype=torch.int32, device=device)
        return Paths(t(hdr), t(pix_first), vt, int(hdr.size // spp), spp)


def encode(E: torch.Tensor, S: torch.Tensor, n: int | None = None, ld_z: int | None = None,
           out: torch.Tensor | None = None) -> torch.Tensor:
    """Codes of the rows of S (rows padded to a multiple of 4 floats) in the
    blocked layout: z = E s (Eq. 4)."""
    _dev(E, S, out)
    k, nE = E.shape
    n = n or nE
    m, ld_s = S.shape
    ld_z = ld_z or latent_width(k)
    if out is None:
        out = torch.empty(m, ld_z, dtype=torch.float32, device=S.device)
    check(load().hc_encode(_ptr(E.contiguous()), k, n, _ptr(S), m, ld_s, _ptr(out), out.stride(0),
                           _stream()), "hc_encode")
    return out


def shade_spectral(paths: Paths, refl: torch.Tensor, illum: torch.Tensor, T: torch.Tensor, n: int,
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """Per-pixel XYZ of the spectral form; refl/illum rows padded to 4 floats."""
    _dev(refl, illum, T, out)
    if out is None:
        out = torch.empty(paths.n_pixels, 3, dtype=torch.float32, device=refl.device)
    A = _lib.SpectralAssets(refl.data_ptr(), refl.shape[0], n, 0, refl.stride(0), illum.data_ptr(),
                            illum.shape[0], 0, illum.stride(0))
    P = paths.c()
    check(load().hc_shade_spectral(C.byref(P), C.byref(A), _ptr(T.contiguous()), _ptr(out), _stream()),
          "hc_shade_spectral")
    return out


def shade_latent(paths: Paths, codes: torch.Tensor, illum_codes: torch.Tensor, k: int,
                 block_first: int = 0, block_count: int | None = None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Latent image (blocked layout) of the latent form.  block_count=None is
    the fused call over all B passes."""
    _dev(codes, illum_codes, out)
    nb = blocks(k)
    block_count = nb - block_first if block_count is None else block_count
    if out is None:
        out = torch.zeros(paths.n_pixels, latent_width(k), dtype=torch.float32, device=codes.device)
    A = _lib.LatentAssets(codes.data_ptr(), codes.shape[0], k, 0, codes.stride(0),
                          illum_codes.data_ptr(), illum_codes.shape[0], 0, illum_codes.stride(0))
    P = paths.c()
    check(load().hc_shade_latent(C.byref(P), C.byref(A), block_first, block_count, _ptr(out),
                                 out.stride(0), _stream()), "hc_shade_latent")
    return out


def shade_latent_xyz(paths: Paths, codes: torch.Tensor, illum_codes: torch.Tensor, M: torch.Tensor,
                     k: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """XYZ of the latent frame in one launch: the pixel means over all B
    passes, decoded with M = decode_matrix(D, T, k)."""
    _dev(codes, illum_codes, M, out)
    if tuple(M.shape) != (3, 3 * blocks(k)) or not M.is_contiguous():
        raise ValueError(f"M must be a contiguous (3, {3 * blocks(k)}) tensor from decode_matrix")
    if out is None:
        out = torch.empty(paths.n_pixels, 3, dtype=torch.float32, device=codes.device)
    A = _lib.LatentAssets(codes.data_ptr(), codes.shape[0], k, 0, codes.stride(0),
                          illum_codes.data_ptr(), illum_codes.shape[0], 0, illum_codes.stride(0))
    P = paths.c()
    check(load().hc_shade_latent_xyz(C.byref(P), C.byref(A), _ptr(M), _ptr(out), _stream()),
          "hc_shade_latent_xyz")
    return out


def decode_matrix(D: torch.Tensor, T: torch.Tensor, k: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """M = T D as 3 rows of 3 * blocks(k) columns (blocked channel order,
    zero past k), the decoder argument of shade_latent_xyz."""
    _dev(D, T, out)
    n = D.shape[0]
    if out is None:
        out = torch.empty(3, 3 * blocks(k), dtype=torch.float32, device=D.device)
    elif tuple(out.shape) != (3, 3 * blocks(k)) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float32 (3, {3 * blocks(k)}) tensor")
    check(load().hc_decode_matrix(_ptr(D.contiguous()), n, k, _ptr(T.contiguous()), _ptr(out), _stream()),
          "hc_decode_matrix")
    return out


def decode_xyz(D: torch.Tensor, T: torch.Tensor, zimg: torch.Tensor, k: int, spectra: bool = False,
               out: torch.Tensor | None = None):
    """XYZ (and optionally decoded spectra) of a blocked latent image."""
    _dev(D, T, zimg, out)
    n = D.shape[0]
    m = zimg.shape[0]
    if out is None:
        out = torch.empty(m, 3, dtype=torch.float32, device=zimg.device)
    sp = torch.empty(m, n, dtype=torch.float32, device=zimg.device) if spectra else None
    check(load().hc_decode_xyz(_ptr(D.contiguous()), n, k, _ptr(T.contiguous()), _ptr(zimg), m,
                               zimg.stride(0), _ptr(out), _ptr(sp), n, _stream()), "hc_decode_xyz")
    return (out, sp) if spectra else out


def check_paths(paths: Paths, n_texels: int, n_illum: int) -> torch.Tensor:
    """Device int64[3]: bad light ids, bad texel ids, bad pixel ranges."""
    counts = torch.empty(3, dtype=torch.int64, device=paths.hdr.device)
    P = paths.c()
    check(load().hc_check_paths(C.byref(P), n_texels, n_illum, _ptr(counts), _stream()),
          "hc_check_paths")
    return counts


def codec_weights(we: torch.Tensor, wd: torch.Tensor, beta: float = 10.0):
    """float32 E = softplus(we), D = softplus(wd) (Eq. 5)."""
    _dev(we, wd)
    k, n = we.shape
    E = torch.empty(k, n, dtype=torch.float32, device=we.device)
    D = torch.empty(n, k, dtype=torch.float32, device=we.device)
    dt = 1 if we.dtype == torch.float64 else 0
    check(load().hc_codec_weights(_ptr(we.contiguous()), _ptr(wd.contiguous()), k, n, dt, beta,
                                  _ptr(E), _ptr(D), _stream()), "hc_codec_weights")
    return E, D


class CodecWorkspace:
    """Scratch memory for codec steps of one shape (kept across steps)."""

    def __init__(self, k: int, n: int, N: int, device):
        self.bytes = int(load().hc_codec_workspace_size(k, n, N))
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)


EQ8_WEIGHTS = (0.5, 0.75, 1.0, 0.5)   # w_e2e, w_rec, w_code, w_col of Eq. 8 (Sec. 4.5)


def codec_step(we, wd, A, B, N: int, lam: float = 1.0, beta: float = 10.0, idx_a=None, idx_b=None,
               loss=None, grad_e=None, grad_d=None, adam: dict | None = None,
               workspace: CodecWorkspace | None = None, objective: str = "l2", T=None,
               weights=EQ8_WEIGHTS, cos_eps: float = 1e-8, draw: dict | None = None,
               static_scratch: bool = False):
    """One loss/gradient (and optional Adam) evaluation on the GPU.

    A, B: (rows, n) tensors of the parameters' dtype; with idx_a/idx_b the
    batch rows are gathered by index; with draw = dict(seed_a, seed_b, ctr0=0,
    step=None) they are drawn on the device: row i of the a-batch is what
    gen_indices(seed_a, N, rows of A, ctr0, step)[i] would be (likewise b),
    with no index arrays.  adam: dict with m_E, v_E, m_D, v_D,
    step (int64 device tensor), lr, beta1, beta2, eps.  objective "l2" is the
    two-term squared error weighted by lam; "eq8" the four-term loss of
    Eq. 8 with `weights` (w_e2e, w_rec, w_code, w_col) and the 3 x n
    colour-matching matrix T (parameters' dtype).  With static_scratch the
    step runs through hc_codec_step_static (no workspace; the library's static
    device array).  Returns the loss tensor.
    """
    _dev(we, wd, A, B)
    k, n = we.shape
    dt = 1 if we.dtype == torch.float64 else 0
    if objective not in ("l2", "eq8"):
        raise ValueError(f"objective must be 'l2' or 'eq8', not {objective!r}")
    eq8 = objective == "eq8"
    if eq8:
        if T is None or tuple(T.shape) != (3, n) or T.dtype != we.dtype or not T.is_contiguous():
            raise ValueError("objective 'eq8' needs a contiguous 3 x n T of the parameters' dtype")
        _dev(T)
    if loss is None:
        loss = torch.empty((), dtype=we.dtype, device=we.device)
    if static_scratch and workspace is not None:
        raise ValueError("static_scratch takes no workspace")
    if not static_scratch:
        workspace = workspace or CodecWorkspace(k, n, N, we.device)
    ad = None
    if adam is not None:
        ad = _lib.Adam(adam["m_E"].data_ptr(), adam["v_E"].data_ptr(), adam["m_D"].data_ptr(),
                       adam["v_D"].data_ptr(), adam["step"].data_ptr(), adam.get("lr", 1e-3),
                       adam.get("beta1", 0.9), adam.get("beta2", 0.999), adam.get("eps", 1e-8))
    w = tuple(float(x) for x in weights) if eq8 else (0.0, 0.0, 0.0, 0.0)
    dr = None
    if draw is not None:
        if idx_a is not None or idx_b is not None:
            raise ValueError("draw excludes idx_a / idx_b")
        step = draw.get("step")
        if step is not None:
            _dev(step)
        dr = _lib.PairDraw(int(draw["seed_a"]), int(draw["seed_b"]), int(draw.get("ctr0", 0)), _ptr(step))
    args = _lib.CodecArgs(
        k, n, dt, _lib.HC_CODEC_EQ8 if eq8 else _lib.HC_CODEC_L2, beta, lam, we.data_ptr(),
        wd.data_ptr(), A.data_ptr(), B.data_ptr(),
        A.stride(0), B.stride(0), A.shape[0], B.shape[0],
        None if idx_a is None else idx_a.data_ptr(), None if idx_b is None else idx_b.data_ptr(),
        N, loss.data_ptr(), None if grad_e is None else grad_e.data_ptr(),
        None if grad_d is None else grad_d.data_ptr(), C.pointer(ad) if ad is not None else None,
        None if static_scratch else workspace.buf.data_ptr(), 0 if static_scratch else workspace.bytes,
        torch.cuda.current_stream().cuda_stream,
        T.data_ptr() if eq8 else None, *w, cos_eps if eq8 else 0.0,
        C.pointer(dr) if dr is not None else None)
    if static_scratch:
        check(load().hc_codec_step_static(C.byref(args)), "hc_codec_step_static")
    else:
        check(load().hc_codec_step(C.byref(args)), "hc_codec_step")
    return loss


def upsample(net: dict, rgb: torch.Tensor, k: int | None = None, precision: str = "f16",
             ld_z: int | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Latent codes (blocked layout) of RGB texels through the upsampling
    network (Sec. 5).  net: float32 device tensors W1 (128 x 3), b1, W2
    (128 x 128), b2, W3 (k x 128), b3; rgb: (m, >= 3) float32.  precision
    "f16" (fp16 matrix-core operands, fp32 accumulation) or "f32"."""
    W = [net[x].contiguous() for x in ("W1", "b1", "W2", "b2", "W3", "b3")]
    _dev(*W, rgb, out)
    if any(w.dtype != torch.float32 for w in W) or rgb.dtype != torch.float32:
        raise ValueError("upsample takes float32 weights and colours")
    k = k or W[4].shape[0]
    if precision not in ("f16", "f32"):
        raise ValueError(f"precision must be 'f16' or 'f32', not {precision!r}")
    m = rgb.shape[0]
    ld_z = ld_z or latent_width(k)
    if out is None:
        out = torch.empty(m, ld_z, dtype=torch.float32, device=rgb.device)
    mlp = _lib.Mlp(k, W[0].shape[0], *(w.data_ptr() for w in W))
    check(load().hc_upsample(C.byref(mlp), _lib.HC_MLP_F16 if precision == "f16" else _lib.HC_MLP_F32,
                             _ptr(rgb), m, rgb.stride(0), _ptr(out), out.stride(0), _stream()),
          "hc_upsample")
    return out


MLP_HIDDEN = 128


def upsample_param_count(k: int) -> int:
    return int(load().hc_upsample_param_count(k, MLP_HIDDEN))


def unpack_mlp(params: torch.Tensor, k: int) -> dict:
    """Views W1, b1, W2, b2, W3, b3 of a packed parameter vector (the layout
    hc_upsample_train_step uses)."""
    h = MLP_HIDDEN
    sizes = [("W1", (h, 3)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (k, h)), ("b3", (k,))]
    out, o = {}, 0
    for name, shape in sizes:
        n = 1
        for d in shape:
            n *= d
        out[name] = params[o:o + n].view(*shape)
        o += n
    if o != params.numel():
        raise ValueError(f"packed parameters hold {params.numel()} values, expected {o}")
    return out


class UpsampleWorkspace:
    def __init__(self, k: int, N: int, device):
        self.bytes = int(load().hc_upsample_train_workspace_size(k, N))
        self.buf = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        self.ptr = self.buf.data_ptr() + off


def upsample_train_step(params: torch.Tensor, rgb: torch.Tensor, z_gt: torch.Tensor, M: torch.Tensor,
                        white, k: int, N: int, idx=None, w_max: float = 0.3, w_col: float = 0.05,
                        loss=None, grad=None, opt: dict | None = None,
                        workspace: UpsampleWorkspace | None = None, draw: dict | None = None):
    """One loss/gradient (and optional AdamW) evaluation of the upsampling
    network's training objective (Sec. 5.2) on the GPU.  params: packed
    float32 vector; rgb (rows, >= 3) and z_gt (rows, blocked layout) float32;
    M (3 x k) = T D; opt: dict with m, v, step (int64 device tensor), lr,
    beta1, beta2, eps, weight_decay, max_grad_norm.  Batch rows: idx, or with
    draw = dict(seed, ctr0=0, step=None) the rows gen_indices(seed, N, rows,
    ctr0, step) would give, drawn inside the step.  Returns the loss tensor."""
    _dev(params, rgb, z_gt, M, idx, grad)
    dr = None
    if draw is not None:
        if idx is not None:
            raise ValueError("draw excludes idx")
        _dev(draw.get("step"))
        dr = _lib.IndexDraw(int(draw["seed"]), int(draw.get("ctr0", 0)), _ptr(draw.get("step")))
    if loss is None:
        loss = torch.empty((), dtype=torch.float32, device=params.device)
    workspace = workspace or UpsampleWorkspace(k, N, params.device)
    o = None
    if opt is not None:
        o = _lib.AdamW(opt["m"].data_ptr(), opt["v"].data_ptr(), opt["step"].data_ptr(),
                       opt.get("lr", 2e-3), opt.get("beta1", 0.9), opt.get("beta2", 0.999),
                       opt.get("eps", 1e-8), opt.get("weight_decay", 1e-5),
                       opt.get("max_grad_norm", 1.0))
    a = _lib.UpsampleTrainArgs(
        k, MLP_HIDDEN, params.data_ptr(), rgb.data_ptr(), rgb.stride(0), z_gt.data_ptr(),
        z_gt.stride(0), rgb.shape[0], _ptr(idx), N, M.contiguous().data_ptr(),
        (C.c_double * 3)(*[float(w) for w in white]), w_max, w_col, loss.data_ptr(), _ptr(grad),
        C.pointer(o) if o is not None else None, workspace.ptr, workspace.bytes, _stream(),
        C.pointer(dr) if dr is not None else None)
    check(load().hc_upsample_train_step(C.byref(a)), "hc_upsample_train_step")
    return loss


def gen_paths(n_pixels: int, spp: int, l_min: int, l_max: int, n_tex: int, n_illum: int, seed: int,
              device="cuda") -> Paths:
    """Generate a frame's records on the GPU (same draws as synth.gen_paths)."""
    g = _lib.PathGen(n_pixels, spp, l_min, l_max, n_illum, n_tex, seed)
    hdr = torch.empty(n_pixels * spp, dtype=torch.int32, device=device)
    pf = torch.empty(n_pixels, dtype=torch.int32, device=device)
    total = torch.empty(1, dtype=torch.int64, device=device)
    wsb = int(load().hc_gen_workspace_size(n_pixels))
    ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=device)
    check(load().hc_gen_path_headers(C.byref(g), _ptr(hdr), _ptr(pf), _ptr(total), _ptr(ws), wsb,
                                     _stream()), "hc_gen_path_headers")
    nv = int(total.item())
    if nv >= 1 << 32:
        raise ValueError(f"{nv} vertex records exceed the 2^32 limit of one frame")
    vtx = torch.empty(nv, 2, dtype=torch.int32, device=device)
    check(load().hc_gen_path_vertices(C.byref(g), _ptr(pf), _ptr(vtx), nv, _stream()),
          "hc_gen_path_vertices")
    return Paths(hdr, pf, vtx, n_pixels, spp)


def gen_indices(seed: int, count: int, n: int, ctr0: int = 0, step: torch.Tensor | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """count uniform indices in [0, n) (same draws as synth.uniform_indices)."""
    dev = step.device if step is not None else "cuda"
    if out is None:
        out = torch.empty(count, dtype=torch.int32, device=dev)
    check(load().hc_gen_indices(seed, ctr0, _ptr(step), count, n, _ptr(out), _stream()),
          "hc_gen_indices")
    return out


def stream_probe(src: torch.Tensor, dst: torch.Tensor, mode: str = "read", grid: int = 2048) -> torch.Tensor:
    """Streaming probe (see hc_stream_probe): mode "read" reads every
    16-byte chunk of src and writes grid * 256 per-lane sums into dst;
    "copy" copies src into dst.  src and dst are contiguous float32."""
    _dev(src, dst)
    if src.numel() % 4 or not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("stream_probe: src must be contiguous with a multiple of 4 floats")
    m = {"read": 0, "copy": 1}[mode]
    need = grid * 256 if m == 0 else src.numel()
    if dst.numel() < need:
        raise ValueError(f"stream_probe: dst holds {dst.numel()} floats, needs {need}")
    check(load().hc_stream_probe(_ptr(src), _ptr(dst), src.numel() // 4, m, grid, _stream()),
          "hc_stream_probe")
    return dst


ALU_PROBE_OPS = ("fma_f32", "exp_f32", "rcp_f32", "exp_f16", "rcp_f16", "pk_fma_f16")
ALU_PROBE_CHAINS, ALU_PROBE_ITERS = 8, 2048   # per lane (HC_ALU_PROBE_CHAINS, HC_ALU_PROBE_ITERS)


def alu_probe(op: str, out: torch.Tensor) -> torch.Tensor:
    """Issue-rate probe (see hc_alu_probe): each of the out.numel() lanes
    (a multiple of 256) issues ALU_PROBE_CHAINS * ALU_PROBE_ITERS
    instructions of kind op (one of ALU_PROBE_OPS) and writes one float."""
    _dev(out)
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() % 256 or out.numel() == 0:
        raise ValueError("alu_probe: out must be contiguous float32 with a positive multiple of 256 elements")
    check(load().hc_alu_probe(ALU_PROBE_OPS.index(op), _ptr(out), out.numel() // 256, _stream()),
          "hc_alu_probe")
    return out


def gather_probe(vtx: torch.Tensor, table: torch.Tensor, row_floats: int, unroll: int = 4,
                 lanes_per_row: int = 1, grid: int = 2048, out: torch.Tensor | None = None) -> torch.Tensor:
    """Random-gather probe over a record stream (see hc_gather_probe): the
    rows the shading kernels gather for these records, read and summed with
    nothing else done.  vtx is (V, 2) 32-bit records, table (rows, ld) float32.
    Returns the grid * 256 per-lane sums."""
    _dev(vtx, table)
    if out is None:
        out = torch.empty(grid * 256, dtype=torch.float32, device=table.device)
    check(load().hc_gather_probe(_ptr(vtx), int(vtx.shape[0]), _ptr(table), int(table.shape[0]),
                                 int(table.stride(0)), row_floats, unroll, lanes_per_row, grid,
                                 _ptr(out), _stream()), "hc_gather_probe")
    return out
