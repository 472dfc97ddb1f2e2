// The per-pixel decode xyz = M z with M = T D (Eq. 4, right; T = T_cmf),
// shared by the decode kernels and the shading kernel's fused epilogue so
// that both give the same bits.  M is 3 rows of 3NB floats in the blocked
// channel order (channel c of block b at column 3b + c), zero past k.
#pragma once

#include "hc_internal.hpp"

namespace hc {

// Entry e of M (row e / 3NB, column e % 3NB): one fused multiply-add per
// spectral sample, in sample order.
template <int NB>
__device__ __forceinline__ float decoder_entry(const float* D, const float* T, int n, int k, int e) {
    const int ch = e / (3 * NB), c = e % (3 * NB);
    float acc = 0.f;
    if (c < k)
        for (int i = 0; i < n; ++i) acc = __builtin_fmaf(T[ch * n + i], D[i * k + c], acc);
    return acc;
}

// x, y, w of one latent pixel z (3NB channels): one fused multiply-add per
// channel, in channel order; padded channels meet M's zero columns.
template <int NB>
__device__ __forceinline__ void decode_dot(const float* M, const float (&z)[3 * NB], float& x, float& y,
                                           float& w) {
    x = 0.f;
    y = 0.f;
    w = 0.f;
#pragma unroll
    for (int c = 0; c < 3 * NB; ++c) {
        x = __builtin_fmaf(M[c], z[c], x);
        y = __builtin_fmaf(M[3 * NB + c], z[c], y);
        w = __builtin_fmaf(M[6 * NB + c], z[c], w);
    }
}

}  // namespace hc
