"""ctypes binding of libhc.so (the C ABI declared in include/hc.h).

Only argument marshalling lives here.  The library is loaded on first use;
if it is missing the import of any operation raises, naming the build step.
"""

from __future__ import annotations

import ctypes as C
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
# HC_LIBRARY names another build of the same library to load (the
# host-sanitized checking build); by default the in-tree libhc.so
LIB_PATH = os.environ.get("HC_LIBRARY") or os.path.join(_PKG, "libhc.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "hc.h")

HC_OK, HC_EINVAL, HC_ESHAPE, HC_EALIGN, HC_ENOMEM, HC_EDEVICE, HC_EUNSUPPORTED = range(7)
HC_CODEC_L2, HC_CODEC_EQ8 = 0, 1
HC_MLP_F32, HC_MLP_F16 = 0, 1
HC_CODEC_STATIC_SCRATCH_BYTES = 16 << 20

vp = C.c_void_p
i32, i64, u64, f64, sz = C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_size_t


class HCError(RuntimeError):
    def __init__(self, status: int, fn: str, detail: str):
        super().__init__(f"{fn} failed with {status_name(status)}: {detail}")
        self.status = status


class Paths(C.Structure):
    _fields_ = [("n_pixels", i64), ("spp", i32), ("reserved0", i32), ("hdr", vp),
                ("pix_first", vp), ("vtx", vp), ("n_vertices", i64)]


class SpectralAssets(C.Structure):
    _fields_ = [("refl", vp), ("n_texels", i64), ("n", i32), ("reserved0", i32), ("ld", i64),
                ("illum", vp), ("n_illum", i32), ("reserved1", i32), ("ld_illum", i64)]


class LatentAssets(C.Structure):
    _fields_ = [("codes", vp), ("n_texels", i64), ("k", i32), ("reserved0", i32), ("ld", i64),
                ("illum_codes", vp), ("n_illum", i32), ("reserved1", i32), ("ld_illum", i64)]


class Adam(C.Structure):
    _fields_ = [("m_E", vp), ("v_E", vp), ("m_D", vp), ("v_D", vp), ("step", vp),
                ("lr", f64), ("beta1", f64), ("beta2", f64), ("eps", f64)]


class PairDraw(C.Structure):
    _fields_ = [("seed_a", u64), ("seed_b", u64), ("ctr0", u64), ("ctr_scale_dev", vp)]


class CodecArgs(C.Structure):
    _fields_ = [("k", i32), ("n", i32), ("dtype", i32), ("objective", i32),
                ("beta", f64), ("lam", f64), ("Wt_E", vp), ("Wt_D", vp), ("A", vp), ("B", vp),
                ("ld_a", i64), ("ld_b", i64), ("rows_a", i64), ("rows_b", i64),
                ("idx_a", vp), ("idx_b", vp), ("N", i64), ("loss", vp), ("grad_E", vp),
                ("grad_D", vp), ("adam", C.POINTER(Adam)), ("workspace", vp),
                ("workspace_bytes", sz), ("stream", vp), ("T", vp), ("w_e2e", f64), ("w_rec", f64),
                ("w_code", f64), ("w_col", f64), ("cos_eps", f64), ("draw", C.POINTER(PairDraw))]


class Mlp(C.Structure):
    _fields_ = [("k", i32), ("hidden", i32), ("W1", vp), ("b1", vp), ("W2", vp), ("b2", vp),
                ("W3", vp), ("b3", vp)]


class AdamW(C.Structure):
    _fields_ = [("m", vp), ("v", vp), ("step", vp), ("lr", f64), ("beta1", f64), ("beta2", f64),
                ("eps", f64), ("weight_decay", f64), ("max_grad_norm", f64)]


class IndexDraw(C.Structure):
    _fields_ = [("seed", u64), ("ctr0", u64), ("ctr_scale_dev", vp)]


class UpsampleTrainArgs(C.Structure):
    _fields_ = [("k", i32), ("hidden", i32), ("params", vp), ("rgb", vp), ("ld_rgb", i64),
                ("z_gt", vp), ("ld_z", i64), ("rows", i64), ("idx", vp), ("N", i64), ("M", vp),
                ("white", f64 * 3), ("w_max", f64), ("w_col", f64), ("loss", vp), ("grad", vp),
                ("opt", C.POINTER(AdamW)), ("workspace", vp), ("workspace_bytes", sz),
                ("stream", vp), ("draw", C.POINTER(IndexDraw))]


class PathGen(C.Structure):
    _fields_ = [("n_pixels", i64), ("spp", i32), ("l_min", i32), ("l_max", i32), ("n_illum", i32),
                ("n_tex", i64), ("seed", u64)]


class Frame(C.Structure):
    _fields_ = [("hdr", vp), ("pix_first", vp), ("vtx", vp), ("n_pixels", i64), ("n_vertices", i64),
                ("spp", i32), ("n_illum", i32), ("tex", vp), ("n_texels", i64), ("ld_tex", i64),
                ("lights", vp), ("ld_lights", i64), ("image", vp), ("ld_image", i64), ("xyz", vp)]


class Tile(C.Structure):
    _fields_ = [("frame", i32), ("reserved0", i32), ("begin", i64), ("end", i64)]


class EncodeJob(C.Structure):
    _fields_ = [("S", vp), ("Z", vp), ("ld_s", i64), ("ld_z", i64), ("begin", i64), ("end", i64)]


_PROTOS = {
    "hc_status_string": (C.c_char_p, [i32]),
    "hc_last_error": (C.c_char_p, []),
    "hc_version": (i32, []),
    "hc_encode": (i32, [vp, i32, i32, vp, i64, i64, vp, i64, vp]),
    "hc_shade_spectral": (i32, [C.POINTER(Paths), C.POINTER(SpectralAssets), vp, vp, vp]),
    "hc_shade_latent": (i32, [C.POINTER(Paths), C.POINTER(LatentAssets), i32, i32, vp, i64, vp]),
    "hc_decode_xyz": (i32, [vp, i32, i32, vp, vp, i64, i64, vp, vp, i64, vp]),
    "hc_shade_latent_xyz": (i32, [C.POINTER(Paths), C.POINTER(LatentAssets), vp, vp, vp]),
    "hc_decode_matrix": (i32, [vp, i32, i32, vp, vp, vp]),
    "hc_check_paths": (i32, [C.POINTER(Paths), i64, i32, vp, vp]),
    "hc_codec_workspace_size": (sz, [i32, i32, i64]),
    "hc_codec_step": (i32, [C.POINTER(CodecArgs)]),
    "hc_codec_step_static": (i32, [C.POINTER(CodecArgs)]),
    "hc_codec_weights": (i32, [vp, vp, i32, i32, i32, f64, vp, vp, vp]),
    "hc_upsample": (i32, [vp, i32, vp, i64, i64, vp, i64, vp]),
    "hc_upsample_param_count": (i64, [i32, i32]),
    "hc_upsample_train_workspace_size": (sz, [i32, i64]),
    "hc_upsample_train_step": (i32, [vp]),
    "hc_shade_latent_tiles": (i32, [vp, i32, vp, vp, i32, i32, i32, vp]),
    "hc_shade_latent_xyz_tiles": (i32, [vp, i32, vp, vp, i32, i32, vp, i32, vp]),
    "hc_shade_spectral_tiles": (i32, [vp, i32, vp, vp, i32, i32, vp, i32, vp]),
    "hc_decode_tiles": (i32, [vp, i32, vp, vp, i32, vp, i32, i32, vp, i32, vp]),
    "hc_encode_jobs": (i32, [vp, vp, i32, vp, i32, i32, i32, vp]),
    "hc_gen_workspace_size": (sz, [i64]),
    "hc_gen_path_headers": (i32, [C.POINTER(PathGen), vp, vp, vp, vp, sz, vp]),
    "hc_gen_path_vertices": (i32, [C.POINTER(PathGen), vp, vp, i64, vp]),
    "hc_gen_indices": (i32, [u64, u64, vp, i64, i64, vp, vp]),
    "hc_gather_probe": (i32, [vp, i64, vp, i64, i64, i32, i32, i32, i32, vp, vp]),
    "hc_stream_probe": (i32, [vp, vp, i64, i32, i32, vp]),
    "hc_alu_probe": (i32, [i32, vp, i32, vp]),
}

_lib = None


def load():
    """The loaded library (ctypes.CDLL); raises if libhc.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2602_18741_amd.build` "
                "(or __graft_entry__.build()); there is no fallback implementation")
        # torch first: the process then has one HIP runtime, the one the
        # caller's streams and tensors belong to, before the library binds it
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_name(status: int) -> str:
    return load().hc_status_string(status).decode()


def check(status: int, fn: str):
    if status != HC_OK:
        raise HCError(status, fn, load().hc_last_error().decode())


def declared_functions(header: str = HEADER):
    """Function names declared in include/hc.h."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hc_[a-z0-9_]+)\s*\(", text)))
