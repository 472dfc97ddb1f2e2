"""The stress shape: 3840 x 2160 px, 64 spp, path length 1..8, 4096^2 x 81
texture, 256 lights, k = 9.  The whole frame is shaded on the GPU in the
benchmark's layout (rows of 96 floats, codes of 16 floats) and 16,384 seeded
pixels are checked against the FP64 oracle in both forms.  The oracle is
given only the texture rows those pixels reach (texel indices renumbered
into that subset), which leaves every product unchanged and keeps it from
converting the whole 16.7 M x 81 table to FP64."""

import numpy as np
import pytest
import torch

import synth
from oracle import shade as osh
from tests.conftest import xyz_close

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_stress_frame_sampled_pixels():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops
    w = synth.workload(4, ld_tex=96)
    spec, n, k = w["paths"], 81, 9
    refl = torch.from_numpy(w["refl"]).cuda()
    illum = ops.padded(torch.from_numpy(w["illum"]).cuda())
    T, E, D = (torch.from_numpy(w[x]).cuda() for x in ("T", "E", "D"))
    P = ops.gen_paths(spec.n_pixels, spec.spp, spec.l_min, spec.l_max, spec.n_tex, spec.n_illum,
                      spec.seed)
    assert P.n_vertices > 2_000_000_000
    xyz_s = ops.shade_spectral(P, refl, illum, T, n)
    codes = ops.encode(E, refl, n=n, out=torch.empty(spec.n_tex, 16, device="cuda"))
    lc = ops.encode(E, illum, n=n, out=torch.empty(spec.n_illum, 16, device="cuda"))
    xyz_l = ops.decode_xyz(D, T, ops.shade_latent(P, codes, lc, k), k)
    torch.cuda.synchronize()
    xs, xl = xyz_s.cpu().numpy(), xyz_l.cpu().numpy()
    # the device records of sampled pixels, among them the frame's last ones
    # (record indices past 2^31), equal the host generator's
    gpix = np.concatenate([np.sort(np.random.default_rng(5).choice(spec.n_pixels - 256, 256, replace=False)),
                           np.arange(spec.n_pixels - 256, spec.n_pixels)])
    gh, gpf, gv = synth.records_of_pixels(spec, gpix)
    pf_dev = P.pix_first[torch.from_numpy(gpix).cuda()].cpu().numpy().view(np.uint32).astype(np.int64)
    assert pf_dev[-1] > 2 ** 31
    counts = (gh >> 24).astype(np.int64).reshape(-1, spec.spp).sum(axis=1)
    rows = np.concatenate([np.arange(f, f + c) for f, c in zip(pf_dev, counts)])
    hdr_rows = (gpix[:, None] * spec.spp + np.arange(spec.spp)[None, :]).ravel()
    assert np.array_equal(P.hdr[torch.from_numpy(hdr_rows).cuda()].cpu().numpy().view(np.uint32), gh)
    assert np.array_equal(P.vtx[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32), gv)
    del P, refl, codes, xyz_s, xyz_l
    torch.cuda.empty_cache()
    pix = np.sort(np.random.default_rng(4).choice(spec.n_pixels, 16384, replace=False))
    hdr, pf, vtx = synth.records_of_pixels(spec, pix)
    used, inv = np.unique(vtx[:, 0], return_inverse=True)
    vsub = vtx.copy()
    vsub[:, 0] = inv.astype(vtx.dtype)
    tex = w["refl"][used, :n]
    assert xyz_close(xs[pix], osh.shade_spectral(hdr, pf, vsub, spec.spp, tex, w["illum"], w["T"]),
                     2e-5, 1e-7) <= 1.0
    z = osh.shade_latent(hdr, pf, vsub, spec.spp, osh.encode(w["E"], tex), osh.encode(w["E"], w["illum"]))
    assert xyz_close(xl[pix], osh.decode(w["D"], w["T"], z)[1], 2e-5, 1e-7) <= 1.0
