"""Writes the stored expected values under tests/golden/ from the FP64
oracle alone (run from the repository root: python tests/golden/make_golden.py).

Each fixture regenerates its inputs from the seeded generators in synth/ and
stores the oracle's outputs, so a later change to the oracle or the
generators shows up as a mismatch (tests/test_golden.py), and the GPU path is
compared with values that no GPU code produced (tests/test_gpu_golden.py).
"""

from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))   # the repository root

import synth  # noqa: E402
from oracle import codec, multibounce, shade, upsample  # noqa: E402


def tiny_frame_inputs():
    """8 x 8 pixels, 4 spp, path length 0..3, 16 reflectances, 6 lights,
    k = 6 with U[0,1] E and D, n = 31."""
    rng = np.random.default_rng([7, 0])
    n, k = 31, 6
    refl = synth.reflectances(rng, n, 16)
    illum = synth.illuminant_table(rng, n, 3, 3, 5.0, 15.0)
    E, D = synth.codec_uniform(np.random.default_rng([7, 3]), k, n)
    spec = synth.PathSpec(n_pixels=64, spp=4, l_min=0, l_max=3, n_tex=16, n_illum=6, seed=7002)
    hdr, pf, vtx = synth.gen_paths(spec)
    return dict(n=n, k=k, refl=refl, illum=illum, E=E, D=D, T=synth.cmf_matrix(n), spec=spec,
                hdr=hdr, pf=pf, vtx=vtx)


def codec_inputs():
    """n = 31, k = 6, 64 pairs, parameters from N(0, 0.1)."""
    rng = np.random.default_rng([7, 4])
    n, k = 31, 6
    we, wd = synth.codec_init(rng, k, n)
    a = synth.reflectances(rng, n, 64)
    b = synth.illuminant_table(rng, n, 32, 32, 5.0, 15.0)
    return dict(n=n, k=k, we=we, wd=wd, a=a, b=b, T=synth.cmf_matrix(n))


def chain_inputs():
    """16 chains of 3 bounces at n = 31, k = 6 (U[0,1] codec)."""
    rng = np.random.default_rng([7, 6])
    n, k, C = 31, 6, 16
    R = synth.reflectances(rng, n, C * 3)
    L = synth.illuminant_table(rng, n, C // 2, C // 2, 5.0, 15.0)
    E, D = synth.codec_uniform(np.random.default_rng([7, 7]), k, n)
    return dict(n=n, k=k, C=C, R=R, L=L, E=E, D=D, T=synth.cmf_matrix(n))


def mlp_inputs():
    """k = 6 network with N(0, 1/fan_in) weights and N(0, 0.3) biases, 32 colours."""
    rng = np.random.default_rng([7, 8])
    h, k = 128, 6
    net = dict(W1=rng.normal(0, 1 / np.sqrt(3), (h, 3)), b1=rng.normal(0, 0.3, h),
               W2=rng.normal(0, 1 / np.sqrt(h), (h, h)), b2=rng.normal(0, 0.3, h),
               W3=rng.normal(0, 1 / np.sqrt(h), (k, h)), b3=rng.normal(0, 0.3, k))
    net = {key: v.astype(np.float32) for key, v in net.items()}
    rgb = rng.uniform(0, 1, (32, 3)).astype(np.float32)
    return dict(k=k, net=net, rgb=rgb)


def compute():
    out = {}
    f = tiny_frame_inputs()
    xs = shade.shade_spectral(f["hdr"], f["pf"], f["vtx"], 4, f["refl"], f["illum"], f["T"])
    z, xl = shade.render_latent_xyz(f["hdr"], f["pf"], f["vtx"], 4, f["refl"], f["illum"], f["E"], f["D"],
                                    f["T"])
    out["tiny_frame"] = {"cites": "spectral pixel: Sec. 3 products, T_cmf of Sec. 4.3, sample mean; "
                                  "latent pixel: Eq. 4, Eq. 6, decode once (Fig. 2b)",
                         "xyz_spectral": xs.tolist(), "latent": z.tolist(), "xyz_latent": xl.tolist()}
    c = codec_inputs()
    L2, ge2, gd2 = codec.loss_and_grad(c["we"], c["wd"], c["a"], c["b"], 1.0, 10.0)
    L8, ge8, gd8 = codec.loss_eq8_and_grad(c["we"], c["wd"], c["a"], c["b"], c["T"])
    out["codec"] = {"cites": "Eq. 5 (softplus weights), Eq. 8 (losses)",
                    "l2": {"loss": L2, "grad_E": ge2.tolist(), "grad_D": gd2.tolist()},
                    "eq8": {"loss": L8, "grad_E": ge8.tolist(), "grad_D": gd8.tolist()}}
    m = chain_inputs()
    x0, xs, xl = multibounce.chain_xyz(m["R"].reshape(m["C"], 3, m["n"]), m["L"], m["E"], m["D"], m["T"])
    out["chains"] = {"cites": "Eq. 10 (multi-bounce chains), Eq. 6", "xyz_light": x0.tolist(),
                     "xyz_spectral": xs.tolist(), "xyz_latent": xl.tolist()}
    u = mlp_inputs()
    out["upsample"] = {"cites": "Sec. 5.1 (three layers, width 128, SiLU)",
                       "z": upsample.upsample(u["net"], u["rgb"]).tolist()}
    return out


def main():
    path = os.path.join(HERE, "oracle_values.json")
    with open(path, "w") as fh:
        json.dump(compute(), fh, indent=1)
        fh.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
