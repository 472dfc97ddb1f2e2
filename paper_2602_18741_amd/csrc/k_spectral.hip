// Spectral form: light-path throughput over n wavelength samples, XYZ by the
// colour-matching matrix, per-pixel sample mean by shuffles.  Every index
// read from the records is clamped to its buffer.

#include "shade_common.hpp"

namespace hc {
namespace {
using namespace shade;

// G lanes per path; a lane owns the float4 chunks c = qq*G + sub (qq < Q) of
// the n samples, so one load instruction covers G consecutive chunks of each
// path's texel row: one 128-byte line for G = 8.  (2 and 4 lanes per path
// measured the same at n = 31.)
constexpr int kSpecLanes = 8;

struct SpectralFrame {
    PathView P;
    const float* refl;
    int64_t ld;
    uint32_t n_tex;
    const float* illum;
    int64_t ld_l;
    uint32_t n_illum;
    int n;
    int nq;  // float4 chunks holding the n samples
    const float* T;
    float* xyz;
    float inv_spp;
};

__device__ __forceinline__ void stage_lights(const SpectralFrame& f, float4* s_light) {
    for (uint32_t i = threadIdx.x; i < f.n_illum * uint32_t(f.nq); i += kBlock) {
        const uint32_t l = i / f.nq, c = i % f.nq;
        s_light[i] = ld4(f.illum + int64_t(l) * f.ld_l + 4 * c);
    }
}

// The calling wave shades pixels [q0, min(q0 + pw, q_end)).  With LDS the
// light spectra come from the staged table s_light, else from global memory.
template <int G, int Q, bool LDS>
__device__ __forceinline__ void spectral_group(const SpectralFrame& f, int64_t q0, int64_t q_end,
                                               const float4* s_light) {
    const PathView& P = f.P;
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane & (G - 1);
    const int slot = lane / G;

    // colour-matching weights of this lane's samples; zero past n
    float4 Tr[3][Q];
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) {
        const int c = qq * G + sub;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float w[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 4 * c + e;
                w[e] = (i < f.n) ? ldg_f32(f.T + ch * f.n + i) : 0.f;
            }
            Tr[ch][qq] = make_float4(w[0], w[1], w[2], w[3]);
        }
    }

    const int seg = P.spp_pad;  // slots per pixel segment
    const int j0 = slot % seg;
    const int64_t q = q0 + slot / seg;
    const bool pix_ok = q < q_end;
    uint32_t next = pix_ok ? ldg_u32(P.pix_first + q) : 0u;
    float ax = 0.f, ay = 0.f, az = 0.f;

    for (int r = 0; r < P.rounds; ++r) {
        const int j = j0 + r * seg;
        const bool live = pix_ok && j < P.spp;
        const uint32_t h = live ? ldg_u32(P.hdr + (q * P.spp + j)) : 0u;
        const uint32_t len = h >> 24;
        uint32_t total;
        const uint32_t first = next + segment_scan(len, j0, seg, G, total);
        next += total;
        if (live) {
            float4 prod[Q];
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) prod[qq] = make_float4(1.f, 1.f, 1.f, 1.f);
            float wprod = 1.f;
            const uint32_t end = (first < P.n_vertices) ? min(first + len, P.n_vertices) : first;
            // U vertices at a time: records, then rows, all in flight before
            // the first multiply; padding slots multiply by 1
            constexpr int U = Q <= 2 ? 4 : 2;
            for (uint32_t jv = first; jv < end; jv += U) {
                // records first, all U in flight: slots past the path read the
                // following (in-bounds) records, which the wave fetches anyway;
                // their weights and rows are replaced by 1 below
                uint2 rec[U];
#pragma unroll
                for (int u = 0; u < U; ++u) rec[u] = ldg_u2(P.vtx + min(jv + u, P.n_vertices - 1u));
                // rows are loaded unconditionally (no branch per vertex): a
                // padding slot reads texel 0's row, which stays in cache, and a
                // lane past the n samples re-reads the row's last chunk; both
                // are replaced by 1 below
                uint32_t tex[U];
                float wt[U];
                bool ok[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    ok[u] = jv + u < end;
                    tex[u] = ok[u] ? min(rec[u].x, f.n_tex - 1u) : 0u;
                    wt[u] = ok[u] ? __uint_as_float(rec[u].y) : 1.f;
                }
                float4 row[U][Q];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const float* rp = f.refl + uint64_t(tex[u]) * uint32_t(f.ld);  // ld < 2^31
#pragma unroll
                    for (int qq = 0; qq < Q; ++qq) {
                        const int c = qq * G + sub;
                        const float4 v = ld4(rp + 4 * min(c, f.nq - 1));
                        row[u][qq] = (ok[u] && c < f.nq) ? v : make_float4(1.f, 1.f, 1.f, 1.f);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int qq = 0; qq < Q; ++qq) prod[qq] = mul4(prod[qq], row[u][qq]);
                    wprod *= wt[u];
                }
            }
            const uint32_t lid = min(h & 0xFFFFFFu, f.n_illum - 1u);
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) {
                const int c = qq * G + sub;
                if (c < f.nq) {
                    const float4 lt = LDS ? s_light[lid * f.nq + c]
                                          : ld4(f.illum + int64_t(lid) * f.ld_l + 4 * c);
                    float4 s = mul4(scale4(lt, wprod), prod[qq]);
                    // samples past n carry no colour weight; drop them so
                    // non-finite row padding cannot leak in
                    if (4 * c + 3 >= f.n) {
                        if (4 * c + 0 >= f.n) s.x = 0.f;
                        if (4 * c + 1 >= f.n) s.y = 0.f;
                        if (4 * c + 2 >= f.n) s.z = 0.f;
                        if (4 * c + 3 >= f.n) s.w = 0.f;
                    }
                    ax += Tr[0][qq].x * s.x + Tr[0][qq].y * s.y + Tr[0][qq].z * s.z + Tr[0][qq].w * s.w;
                    ay += Tr[1][qq].x * s.x + Tr[1][qq].y * s.y + Tr[1][qq].z * s.z + Tr[1][qq].w * s.w;
                    az += Tr[2][qq].x * s.x + Tr[2][qq].y * s.y + Tr[2][qq].z * s.z + Tr[2][qq].w * s.w;
                }
            }
        }
    }
    // reduce over the G sample lanes, then over the pixel's slots
    const int span = G * seg;
    for (int m = 1; m < span; m <<= 1) {
        ax += shfl_xor(ax, m);
        ay += shfl_xor(ay, m);
        az += shfl_xor(az, m);
    }
    if (pix_ok && sub == 0 && j0 == 0) {
        float* out = f.xyz + q * 3;
        stg_f32(out + 0, ax * f.inv_spp);
        stg_f32(out + 1, ay * f.inv_spp);
        stg_f32(out + 2, az * f.inv_spp);
    }
}

template <int G, int Q>
__global__ __launch_bounds__(kBlock) void shade_spectral_kernel(SpectralFrame f, int lights_in_lds) {
    extern __shared__ float4 s_light[];
    if (lights_in_lds) {
        stage_lights(f, s_light);
        __syncthreads();
    }
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    const int64_t q0 = wave * f.P.pw;
    if (q0 >= f.P.n_pixels) return;
    if (lights_in_lds)
        spectral_group<G, Q, true>(f, q0, f.P.n_pixels, s_light);
    else
        spectral_group<G, Q, false>(f, q0, f.P.n_pixels, s_light);
}

// Persistent launch over a tile table (see the latent form).
template <int G, int Q>
__global__ __launch_bounds__(kBlock) void shade_spectral_tiles_kernel(const hc_frame* __restrict__ frames,
                                                                      int n_frames,
                                                                      const hc_tile* __restrict__ tiles,
                                                                      const int32_t* __restrict__ n_tiles_dev,
                                                                      int max_tiles, int n,
                                                                      const float* __restrict__ T) {
    extern __shared__ float4 s_light[];
    const int n_tiles = min(*n_tiles_dev, max_tiles);
    const int wave = wave_in_block();
    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        int64_t begin, end;
        const hc_tile tile = tiles[t];
        if (!tile_range(tile, frames, n_frames, begin, end)) continue;
        const hc_frame& fr = frames[tile.frame];
        SpectralFrame f;
        f.P = make_view(fr.hdr, fr.pix_first, fr.vtx, fr.n_pixels, fr.n_vertices, fr.spp, kWave / G);
        f.refl = fr.tex;
        f.ld = fr.ld_tex;
        f.n_tex = static_cast<uint32_t>(fr.n_texels);
        f.illum = fr.lights;
        f.ld_l = fr.ld_lights;
        f.n_illum = static_cast<uint32_t>(fr.n_illum);
        f.n = n;
        f.nq = (n + 3) / 4;
        f.T = T;
        f.xyz = fr.xyz;
        f.inv_spp = 1.0f / static_cast<float>(fr.spp);
        const bool lds = size_t(f.n_illum) * f.nq * sizeof(float4) <= kLightLdsBytes;
        __syncthreads();
        if (lds) stage_lights(f, s_light);
        __syncthreads();
        const int64_t groups = (end - begin + f.P.pw - 1) / f.P.pw;
        for (int64_t g = wave; g < groups; g += kWavesPerBlock) {
            if (lds)
                spectral_group<G, Q, true>(f, begin + g * f.P.pw, end, s_light);
            else
                spectral_group<G, Q, false>(f, begin + g * f.P.pw, end, s_light);
        }
    }
}

template <int G, int Q>
hc_status launch_spectral_gq(const SpectralFrame& f, int lights_in_lds, int64_t blocks, size_t lds,
                             hipStream_t st) {
    hipLaunchKernelGGL((shade_spectral_kernel<G, Q>), dim3(uint32_t(blocks)), dim3(kBlock), lds, st, f,
                       lights_in_lds);
    return launch_status("hc_shade_spectral");
}

template <int G, int Q>
hc_status launch_spectral_tiles_gq(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                   const int32_t* n_tiles, int max_tiles, int n, const float* T, int grid,
                                   hipStream_t st) {
    hipLaunchKernelGGL((shade_spectral_tiles_kernel<G, Q>), dim3(grid), dim3(kBlock), kLightLdsBytes, st,
                       frames, n_frames, tiles, n_tiles, max_tiles, n, T);
    return launch_status("hc_shade_spectral_tiles");
}

}  // namespace

hc_status launch_shade_spectral(const hc_paths& P, const hc_spectral_assets& A, const float* T,
                                float* xyz, hipStream_t st) {
    SpectralFrame f;
    f.P = make_view(P, kWave / kSpecLanes);
    f.refl = A.refl;
    f.ld = A.ld;
    f.n_tex = static_cast<uint32_t>(A.n_texels);
    f.illum = A.illum;
    f.ld_l = A.ld_illum;
    f.n_illum = static_cast<uint32_t>(A.n_illum);
    f.n = A.n;
    f.nq = static_cast<int>(ceil_div(A.n, 4));
    f.T = T;
    f.xyz = xyz;
    f.inv_spp = 1.0f / static_cast<float>(P.spp);
    const size_t lds_need = size_t(A.n_illum) * f.nq * sizeof(float4);
    const int lights_in_lds = lds_need <= kLightLdsBytes;
    const size_t lds = lights_in_lds ? lds_need : 0;
    const int64_t waves = ceil_div(P.n_pixels, f.P.pw);
    const int64_t blocks = ceil_div(waves, kWavesPerBlock);
    if (blocks > 0x7FFFFFFF) {
        set_error("hc_shade_spectral: frame too large for one launch");
        return HC_ESHAPE;
    }
    switch (ceil_div(f.nq, kSpecLanes)) {
        case 1: return launch_spectral_gq<kSpecLanes, 1>(f, lights_in_lds, blocks, lds, st);
        case 2: return launch_spectral_gq<kSpecLanes, 2>(f, lights_in_lds, blocks, lds, st);
        case 3: return launch_spectral_gq<kSpecLanes, 3>(f, lights_in_lds, blocks, lds, st);
        case 4: return launch_spectral_gq<kSpecLanes, 4>(f, lights_in_lds, blocks, lds, st);
        default:
            set_error("hc_shade_spectral: n=%d unsupported", A.n);
            return HC_EUNSUPPORTED;
    }
}

hc_status launch_shade_spectral_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                      const int32_t* n_tiles, int max_tiles, int n, const float* T,
                                      int grid, hipStream_t st) {
    switch (ceil_div(ceil_div(n, 4), kSpecLanes)) {
        case 1: return launch_spectral_tiles_gq<kSpecLanes, 1>(frames, n_frames, tiles, n_tiles, max_tiles, n, T, grid, st);
        case 2: return launch_spectral_tiles_gq<kSpecLanes, 2>(frames, n_frames, tiles, n_tiles, max_tiles, n, T, grid, st);
        case 3: return launch_spectral_tiles_gq<kSpecLanes, 3>(frames, n_frames, tiles, n_tiles, max_tiles, n, T, grid, st);
        case 4: return launch_spectral_tiles_gq<kSpecLanes, 4>(frames, n_frames, tiles, n_tiles, max_tiles, n, T, grid, st);
        default:
            set_error("hc_shade_spectral_tiles: n=%d unsupported", n);
            return HC_EUNSUPPORTED;
    }
}

}  // namespace hc
