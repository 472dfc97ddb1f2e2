"""The C-ABI library loads, exports every declared function, and rejects
bad arguments on the host before touching the GPU (no compute calls)."""

import ctypes as C

import pytest

from paper_2602_18741_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_function_is_exported(lib):
    names = _lib.declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib._PROTOS, f"{name} has no ctypes prototype"


def test_status_strings(lib):
    assert _lib.status_name(_lib.HC_OK) == "HC_OK"
    assert _lib.status_name(_lib.HC_ESHAPE) == "HC_ESHAPE"
    assert _lib.status_name(99) == "HC_UNKNOWN"
    assert lib.hc_version() >= 100


def test_struct_sizes_match_header():
    # sizes implied by include/hc.h on LP64
    assert C.sizeof(_lib.Paths) == 48
    assert C.sizeof(_lib.SpectralAssets) == 56
    assert C.sizeof(_lib.LatentAssets) == 56
    assert C.sizeof(_lib.Adam) == 72
    assert C.sizeof(_lib.PathGen) == 40
    assert C.sizeof(_lib.PairDraw) == 32
    assert C.sizeof(_lib.CodecArgs) == 232
    assert C.sizeof(_lib.IndexDraw) == 24
    assert C.sizeof(_lib.UpsampleTrainArgs) == 176


def _err(status):
    return status, _lib.load().hc_last_error().decode()


def test_encode_rejects_bad_shapes(lib):
    s, msg = _err(lib.hc_encode(None, 0, 31, None, 10, 32, None, 8, None))
    assert s == _lib.HC_ESHAPE and "k=0" in msg
    s, msg = _err(lib.hc_encode(None, 6, 129, None, 10, 132, None, 8, None))
    assert s == _lib.HC_ESHAPE
    s, msg = _err(lib.hc_encode(None, 6, 31, None, 10, 31, None, 8, None))
    assert s == _lib.HC_ESHAPE and "ld_s" in msg
    s, msg = _err(lib.hc_encode(None, 6, 31, None, 10, 32, None, 6, None))
    assert s == _lib.HC_ESHAPE and "ld_z" in msg
    s, msg = _err(lib.hc_encode(None, 6, 31, None, 10, 32, None, 8, None))
    assert s == _lib.HC_EINVAL
    # misaligned pointers (never dereferenced: the check comes first)
    s, msg = _err(lib.hc_encode(C.c_void_p(0x1000), 6, 31, C.c_void_p(0x1004), 10, 32,
                                C.c_void_p(0x2000), 8, None))
    assert s == _lib.HC_EALIGN
    # an empty batch is a valid no-op
    assert lib.hc_encode(None, 6, 31, None, 0, 32, None, 8, None) == _lib.HC_OK


def test_shade_rejects_bad_records(lib):
    P = _lib.Paths(10, 0, 0, None, None, None, 0)
    A = _lib.SpectralAssets(None, 1, 31, 0, 32, None, 1, 0, 32)
    s, msg = _err(lib.hc_shade_spectral(C.byref(P), C.byref(A), None, None, None))
    assert s == _lib.HC_ESHAPE and "spp" in msg
    P = _lib.Paths(10, 4, 0, None, None, None, 0)
    s, msg = _err(lib.hc_shade_spectral(C.byref(P), C.byref(A), None, None, None))
    assert s == _lib.HC_EINVAL
    P = _lib.Paths(10, 4, 0, 0x1000, 0x1000, 0x1004, 5)
    L = _lib.LatentAssets(0x1000, 4, 6, 0, 8, 0x1000, 2, 0, 8)
    s, msg = _err(lib.hc_shade_latent(C.byref(P), C.byref(L), 0, 2, C.c_void_p(0x1000), 8, None))
    assert s == _lib.HC_EALIGN and "vtx" in msg
    P = _lib.Paths(10, 4, 0, 0x1000, 0x1000, 0x1000, 5)
    s, msg = _err(lib.hc_shade_latent(C.byref(P), C.byref(L), 1, 2, C.c_void_p(0x1000), 8, None))
    assert s == _lib.HC_ESHAPE and "blocks" in msg
    P = _lib.Paths(0, 4, 0, None, None, None, 0)
    assert lib.hc_shade_latent(C.byref(P), C.byref(L), 0, 2, None, 8, None) == _lib.HC_OK
    # spectral row strides must stay below 2^30 floats (4 GiB per row)
    P = _lib.Paths(10, 4, 0, 0x1000, 0x1000, 0x1000, 5)
    A = _lib.SpectralAssets(0x1000, 1, 31, 0, 1 << 30, 0x1000, 1, 0, 32)
    s, msg = _err(lib.hc_shade_spectral(C.byref(P), C.byref(A), C.c_void_p(0x1000), C.c_void_p(0x1000), None))
    assert s == _lib.HC_ESHAPE and "2^30" in msg


def test_codec_step_rejects_small_workspace(lib):
    need = lib.hc_codec_workspace_size(6, 31, 65536)
    assert need > 0
    args = _lib.CodecArgs(6, 31, 0, 0, 10.0, 1.0, 0x1000, 0x1000, 0x1000, 0x1000, 31, 31,
                          65536, 65536, None, None, 65536, 0x1000, None, None, None,
                          0x1000, need - 8, None)
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_ENOMEM and str(need) in msg
    args.dtype = 2
    assert lib.hc_codec_step(C.byref(args)) == _lib.HC_EINVAL


def test_codec_step_validates_the_pair_draw(lib):
    need = lib.hc_codec_workspace_size(6, 31, 65536)
    args = _lib.CodecArgs(6, 31, 0, 0, 10.0, 1.0, 0x1000, 0x1000, 0x1000, 0x1000, 31, 31,
                          1 << 20, 1 << 20, 0x1000, None, 65536, 0x1000, None, None, None,
                          0x1000, need, None)
    dr = _lib.PairDraw(1, 2, 0, None)
    args.draw = C.pointer(dr)
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_EINVAL and "draw excludes" in msg
    args.idx_a = None
    args.rows_b = 1 << 32
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_ESHAPE and "2^32" in msg
    args.rows_b = 0
    assert lib.hc_codec_step(C.byref(args)) == _lib.HC_ESHAPE
    args.rows_b = 1 << 20
    dr.ctr_scale_dev = 0x1004
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_EALIGN and "counter" in msg


def test_codec_step_validates_the_eq8_objective(lib):
    need = lib.hc_codec_workspace_size(6, 31, 65536)
    args = _lib.CodecArgs(6, 31, 0, 0, 10.0, 1.0, 0x1000, 0x1000, 0x1000, 0x1000, 31, 31,
                          65536, 65536, None, None, 65536, 0x1000, None, None, None,
                          0x1000, need, None)
    args.objective = 7
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_EINVAL and "objective" in msg
    args.objective = _lib.HC_CODEC_EQ8
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_EINVAL and "needs T" in msg
    args.T, args.w_e2e, args.w_rec, args.w_code, args.w_col, args.cos_eps = 0x1000, 0.5, 0.75, 1, -0.5, 1e-8
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_EINVAL and "weights" in msg
    args.w_col, args.cos_eps = float("nan"), 1e-8
    assert lib.hc_codec_step(C.byref(args)) == _lib.HC_EINVAL
    args.w_col, args.cos_eps = 0.5, 0.0
    s, msg = _err(lib.hc_codec_step(C.byref(args)))
    assert s == _lib.HC_EINVAL and "cos_eps" in msg
    args.cos_eps = 1e-8
    args.T = 0x1002                      # misaligned for float32
    assert lib.hc_codec_step(C.byref(args)) == _lib.HC_EALIGN


def test_workspace_covers_both_objectives(lib):
    """The workspace size is the larger of the two objectives' needs: it
    never shrinks as N grows and is at least the partial-row table of the
    float64 plan."""
    for k, n in ((6, 31), (9, 81), (48, 128)):
        sizes = [lib.hc_codec_workspace_size(k, n, N) for N in (1, 7, 64, 4099, 65536, 1 << 20)]
        assert sizes == sorted(sizes) and sizes[0] > 0


def test_gen_rejects_bad_lengths(lib):
    g = _lib.PathGen(16, 4, 3, 2, 8, 64, 1)
    s, msg = _err(lib.hc_gen_path_headers(C.byref(g), None, None, None, None, 0, None))
    assert s == _lib.HC_ESHAPE and "l_min" in msg


def test_upsample_validates_before_launch(lib):
    net = _lib.Mlp(6, 128, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    args = lambda prec=0, m=16, ld_rgb=3, ld_z=8: (C.byref(net), prec, 0x1000, m, ld_rgb, 0x1000, ld_z, None)  # noqa: E731
    net.hidden = 64
    s, msg = _err(lib.hc_upsample(*args()))
    assert s == _lib.HC_EUNSUPPORTED and "hidden" in msg
    net.hidden, net.k = 128, 0
    assert lib.hc_upsample(*args()) == _lib.HC_ESHAPE
    net.k = 49
    assert lib.hc_upsample(*args()) == _lib.HC_ESHAPE
    net.k = 6
    assert lib.hc_upsample(*args(prec=2)) == _lib.HC_EINVAL
    assert lib.hc_upsample(*args(ld_rgb=2)) == _lib.HC_ESHAPE
    assert lib.hc_upsample(*args(ld_z=7)) == _lib.HC_ESHAPE
    assert lib.hc_upsample(*args(m=-1)) == _lib.HC_ESHAPE
    net.W2 = None
    assert lib.hc_upsample(*args()) == _lib.HC_EINVAL
    # an empty input enqueues nothing and needs no buffers
    assert lib.hc_upsample(C.byref(net), 0, None, 0, 3, None, 8, None) == _lib.HC_OK
    net.W2 = 0x1002
    assert lib.hc_upsample(*args()) == _lib.HC_EALIGN


def test_upsample_train_step_validates_the_index_draw(lib):
    need = lib.hc_upsample_train_workspace_size(6, 1024)
    args = _lib.UpsampleTrainArgs(6, 128, 0x1000, 0x1000, 4, 0x1000, 8, 1 << 16, 0x1000, 1024, 0x1000,
                                  (C.c_double * 3)(0.95, 1.0, 1.09), 0.3, 0.05, 0x1000, None, None,
                                  0x10000, need, None)
    dr = _lib.IndexDraw(7, 0, None)
    args.draw = C.pointer(dr)
    s, msg = _err(lib.hc_upsample_train_step(C.byref(args)))
    assert s == _lib.HC_EINVAL and "draw excludes idx" in msg
    args.idx = None
    args.rows = 1 << 32
    s, msg = _err(lib.hc_upsample_train_step(C.byref(args)))
    assert s == _lib.HC_ESHAPE and "2^32" in msg
    args.rows = 1 << 16
    dr.ctr_scale_dev = 0x1004
    s, msg = _err(lib.hc_upsample_train_step(C.byref(args)))
    assert s == _lib.HC_EALIGN and "counter" in msg


def test_gather_probe_rejects_bad_arguments(lib):
    p = C.c_void_p(0x1000)
    s, msg = _err(lib.hc_gather_probe(p, 10, p, 4, 8, 8, 3, 1, 4, p, None))
    assert s == _lib.HC_EINVAL and "unroll" in msg
    s, msg = _err(lib.hc_gather_probe(p, 10, p, 4, 8, 8, 4, 2, 4, p, None))
    assert s == _lib.HC_EINVAL and "lanes_per_row" in msg
    s, msg = _err(lib.hc_gather_probe(p, 10, p, 4, 32, 20, 4, 1, 4, p, None))
    assert s == _lib.HC_ESHAPE and "row_floats" in msg
    s, msg = _err(lib.hc_gather_probe(p, 10, p, 4, 6, 6, 4, 1, 4, p, None))
    assert s == _lib.HC_ESHAPE and "ld" in msg
    s, msg = _err(lib.hc_gather_probe(p, 10, p, 4, 8, 8, 4, 1, 0, p, None))
    assert s == _lib.HC_ESHAPE and "grid" in msg
    s, msg = _err(lib.hc_gather_probe(p, 10, C.c_void_p(0x1004), 4, 8, 8, 4, 1, 4, p, None))
    assert s == _lib.HC_EALIGN
    s, msg = _err(lib.hc_gather_probe(p, 10, None, 4, 8, 8, 4, 1, 4, p, None))
    assert s == _lib.HC_EINVAL


def test_codec_step_static_rejects_a_workspace_and_oversized_shapes(lib):
    """The entry point without allocation takes no workspace, and refuses a
    shape whose step needs more scratch than its static array, before any
    device call."""
    args = _lib.CodecArgs(6, 31, 0, 0, 10.0, 1.0, 0x1000, 0x1000, 0x1000, 0x1000, 31, 31,
                          65536, 65536, None, None, 65536, 0x1000, None, None, None,
                          0x1000, 4096, None)
    s, msg = _err(lib.hc_codec_step_static(C.byref(args)))
    assert s == _lib.HC_EINVAL and "no workspace" in msg
    args.workspace, args.workspace_bytes = None, 0
    args.k, args.n, args.dtype, args.ld_a, args.ld_b = 48, 128, 1, 128, 128
    s, msg = _err(lib.hc_codec_step_static(C.byref(args)))
    assert s == _lib.HC_ENOMEM and str(_lib.HC_CODEC_STATIC_SCRATCH_BYTES) in msg
    args.k = 0
    assert lib.hc_codec_step_static(C.byref(args)) == _lib.HC_ESHAPE


def test_server_table_dtypes_match_the_abi_structs():
    """The server writes its tile and encode-job tables as numpy records;
    their layout is the C structs' (hc_tile, hc_encode_job)."""
    from paper_2602_18741_amd.serve import GpuBackend
    for dt, st in ((GpuBackend._TILE_DT, _lib.Tile), (GpuBackend._JOB_DT, _lib.EncodeJob)):
        assert dt.itemsize == C.sizeof(st)
        for name, _ in st._fields_:
            want = "pad" if name == "reserved0" else name
            assert dt.fields[want][1] == getattr(st, name).offset, name


def test_stream_probe_rejects_bad_arguments(lib):
    p = C.c_void_p(0x1000)
    s, msg = _err(lib.hc_stream_probe(p, p, 16, 2, 4, None))
    assert s == _lib.HC_EINVAL and "mode" in msg
    s, msg = _err(lib.hc_stream_probe(p, p, 16, 0, 0, None))
    assert s == _lib.HC_ESHAPE and "grid" in msg
    s, msg = _err(lib.hc_stream_probe(C.c_void_p(0x1004), p, 16, 1, 4, None))
    assert s == _lib.HC_EALIGN
    s, msg = _err(lib.hc_stream_probe(p, C.c_void_p(0x1004), 16, 1, 4, None))
    assert s == _lib.HC_EALIGN
    s, msg = _err(lib.hc_stream_probe(None, p, 16, 0, 4, None))
    assert s == _lib.HC_EINVAL
    # an empty copy enqueues nothing
    assert lib.hc_stream_probe(None, p, 0, 1, 4, None) == _lib.HC_OK


def test_alu_probe_rejects_bad_arguments(lib):
    p = C.c_void_p(0x1000)
    for op in (-1, 6):
        s, msg = _err(lib.hc_alu_probe(op, p, 4, None))
        assert s == _lib.HC_EINVAL and "op" in msg
    s, msg = _err(lib.hc_alu_probe(0, p, 0, None))
    assert s == _lib.HC_ESHAPE and "grid" in msg
    s, msg = _err(lib.hc_alu_probe(0, None, 4, None))
    assert s == _lib.HC_EINVAL
    s, msg = _err(lib.hc_alu_probe(0, C.c_void_p(0x1002), 4, None))
    assert s == _lib.HC_EALIGN


def test_alu_probe_constants_match_the_header():
    """The binding's chain and iteration counts (which turn the probe's time
    into cycles per instruction) are the header's, and its op order is the
    header's list."""
    import os
    import re
    from paper_2602_18741_amd import ops
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hc.h")).read()
    assert int(re.search(r"#define HC_ALU_PROBE_CHAINS (\d+)", hdr).group(1)) == ops.ALU_PROBE_CHAINS
    assert int(re.search(r"#define HC_ALU_PROBE_ITERS (\d+)", hdr).group(1)) == ops.ALU_PROBE_ITERS
    doc = re.search(r"op  0 fp32 multiply-add, 1 v_exp_f32, 2 v_rcp_f32, 3 v_exp_f16,\s+\*\s+4 v_rcp_f16, 5 packed fp16", hdr)
    assert doc is not None
    assert ops.ALU_PROBE_OPS == ("fma_f32", "exp_f32", "rcp_f32", "exp_f16", "rcp_f16", "pk_fma_f16")


def test_fused_latent_frame_and_decode_matrix_validate(lib):
    P = _lib.Paths(10, 4, 0, 0x1000, 0x1000, 0x1000, 5)
    L = _lib.LatentAssets(0x1000, 4, 6, 0, 8, 0x1000, 2, 0, 8)
    M, xyz = C.c_void_p(0x2000), C.c_void_p(0x3000)
    s, msg = _err(lib.hc_shade_latent_xyz(C.byref(P), C.byref(L), None, xyz, None))
    assert s == _lib.HC_EINVAL and "NULL" in msg
    s, msg = _err(lib.hc_shade_latent_xyz(C.byref(P), C.byref(L), C.c_void_p(0x2002), xyz, None))
    assert s == _lib.HC_EALIGN and "M/xyz" in msg
    s, msg = _err(lib.hc_shade_latent_xyz(C.byref(P), C.byref(L), M, C.c_void_p(0x3001), None))
    assert s == _lib.HC_EALIGN
    s, msg = _err(lib.hc_shade_latent_xyz(C.byref(P), C.byref(_lib.LatentAssets(0x1000, 4, 49, 0, 68, 0x1000, 2,
                                                                                  0, 68)), M, xyz, None))
    assert s == _lib.HC_ESHAPE and "k=49" in msg
    s, msg = _err(lib.hc_shade_latent_xyz(C.byref(P), C.byref(_lib.LatentAssets(0x1000, 4, 6, 0, 4, 0x1000, 2,
                                                                                  0, 8)), M, xyz, None))
    assert s == _lib.HC_ESHAPE and "ld" in msg
    s, msg = _err(lib.hc_shade_latent_xyz(C.byref(_lib.Paths(10, 4, 0, 0x1000, 0x1000, 0x1004, 5)), C.byref(L),
                                          M, xyz, None))
    assert s == _lib.HC_EALIGN and "vtx" in msg
    # an empty frame is a valid no-op, whatever the pointers
    assert lib.hc_shade_latent_xyz(C.byref(_lib.Paths(0, 4, 0, None, None, None, 0)), C.byref(L), None, None,
                                   None) == _lib.HC_OK
    s, msg = _err(lib.hc_decode_matrix(M, 31, 0, M, M, None))
    assert s == _lib.HC_ESHAPE and "k=0" in msg
    s, msg = _err(lib.hc_decode_matrix(M, 0, 6, M, M, None))
    assert s == _lib.HC_ESHAPE and "n=0" in msg
    s, msg = _err(lib.hc_decode_matrix(M, 31, 6, None, M, None))
    assert s == _lib.HC_EINVAL
    s, msg = _err(lib.hc_decode_matrix(M, 31, 6, M, C.c_void_p(0x2002), None))
    assert s == _lib.HC_EALIGN


def test_fused_latent_tiles_validate(lib):
    T = C.c_void_p(0x1000)
    s, msg = _err(lib.hc_shade_latent_xyz_tiles(T, 1, T, T, 16, 6, None, 0, None))
    assert s == _lib.HC_EINVAL and "M" in msg
    s, msg = _err(lib.hc_shade_latent_xyz_tiles(T, 1, T, T, 16, 6, C.c_void_p(0x2002), 0, None))
    assert s == _lib.HC_EINVAL
    s, msg = _err(lib.hc_shade_latent_xyz_tiles(T, 1, T, T, 16, 0, T, 0, None))
    assert s == _lib.HC_ESHAPE and "k=0" in msg
    s, msg = _err(lib.hc_shade_latent_xyz_tiles(None, 1, T, T, 16, 6, T, 0, None))
    assert s == _lib.HC_EINVAL and "table" in msg
    s, msg = _err(lib.hc_shade_latent_xyz_tiles(T, 1, T, T, 16, 6, T, 70000, None))
    assert s == _lib.HC_ESHAPE and "grid" in msg
