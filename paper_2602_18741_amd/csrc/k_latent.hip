// Latent form: light-path throughput in code space.  One lane per path; a
// pixel's paths are contiguous lanes (spp padded to a power of two up to 64,
// larger spp loops over rounds of 64 paths).  Per vertex a lane gathers the
// 16-byte blocks of the texel's code (blocked RGBx layout) and multiplies
// them into its product, block by block (the blockwise Hadamard product);
// the light code comes from LDS when the table fits; the per-pixel sample
// mean is an xor butterfly across the pixel's lanes.  Every index read from
// the records is clamped to its buffer.
//
// Two launches share the per-wave code: one frame per launch, or a fixed
// grid walking a tile table that spans many frames (serving).  The frame
// launch can also decode each pixel's mean to XYZ in its epilogue (M = T D
// staged in LDS beside the light codes), writing 12 bytes per pixel instead
// of the latent row.

#include "decode_common.hpp"
#include "shade_common.hpp"

namespace hc {
namespace {
using namespace shade;

struct LatentFrame {
    PathView P;
    const float* codes;
    int64_t ld;
    uint32_t n_tex;
    const float* lcodes;
    int64_t ld_l;
    uint32_t n_illum;
    int block_first;
    float* zimg;
    int64_t ld_z;
    float inv_spp;
    const float* M;  // fused decode: 3 x 3NB decoder matrix, xyz output
    float* xyz;
};

// Stage the light codes of blocks [block_first, block_first + NB) in LDS.
template <int NB>
__device__ __forceinline__ void stage_lights(const LatentFrame& f, float4* s_light) {
    for (uint32_t i = threadIdx.x; i < f.n_illum * NB; i += kBlock) {
        const uint32_t l = i / NB, b = i % NB;
        s_light[i] = ld4(f.lcodes + int64_t(l) * f.ld_l + 4 * (f.block_first + int(b)));
    }
}

// The calling wave shades pixels [q0, min(q0 + pw, q_end)).  With LDS the
// light codes come from the staged table s_light, else from global memory.
// With XYZ the pixel mean is decoded with the staged decoder matrix s_M.
template <int NB, bool LDS, bool FAR = false, bool XYZ = false>
__device__ __forceinline__ void latent_group(const LatentFrame& f, int64_t q0, int64_t q_end,
                                             const float4* s_light, const float* s_M = nullptr) {
#pragma clang fp contract(off)
    const PathView& P = f.P;
    const int lane = threadIdx.x & (kWave - 1);
    const int seg = P.spp_pad;  // lanes per pixel segment
    const int j0 = lane % seg;
    const int64_t q = q0 + lane / seg;
    const bool pix_ok = q < q_end;
    uint32_t next = pix_ok ? ldg_u32(P.pix_first + q) : 0u;

    float4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = make_float4(0.f, 0.f, 0.f, 0.f);

    for (int r = 0; r < P.rounds; ++r) {
        const int j = j0 + r * seg;
        const bool live = pix_ok && j < P.spp;
        const uint32_t h = live ? ldg_u32(P.hdr + (q * P.spp + j)) : 0u;
        const uint32_t len = h >> 24;
        uint32_t total;
        const uint32_t first = next + segment_scan(len, j0, seg, 1, total);
        next += total;
        if (live) {
            float4 prod[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) prod[b] = make_float4(1.f, 1.f, 1.f, 1.f);
            float wprod = 1.f;
            // vertices past the record array are skipped
            const uint32_t end = (first < P.n_vertices) ? min(first + len, P.n_vertices) : first;
            // U vertices at a time: all record loads, then all row gathers, are
            // in flight before the first multiply; padding slots multiply by 1
            // (FAR: a table past the cache, served from HBM, where fewer
            // requests in flight per lane are served faster)
            constexpr int U0 = NB <= 4 ? 4 : (NB <= 8 ? 2 : 1);
            constexpr int U = FAR && U0 > 1 ? U0 / 2 : U0;
            for (uint32_t jv = first; jv < end; jv += U) {
                // records first, all U in flight: slots past the path read the
                // following (in-bounds) records, which the wave fetches anyway;
                // their weights and rows are replaced by 1 below
                uint2 rec[U];
#pragma unroll
                for (int u = 0; u < U; ++u) rec[u] = ldg_u2(P.vtx + min(jv + u, P.n_vertices - 1u));
                uint32_t tex[U];
                float wt[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    tex[u] = min(rec[u].x, f.n_tex - 1u);
                    wt[u] = (jv + u < end) ? __uint_as_float(rec[u].y) : 1.f;
                }
                float4 row[U][NB];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const float* rp = f.codes + uint64_t(tex[u]) * uint32_t(f.ld) + 4 * f.block_first;  // ld < 2^31
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        row[u][b] = (jv + u < end) ? ld4(rp + 4 * b) : make_float4(1.f, 1.f, 1.f, 1.f);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) prod[b] = mul4(prod[b], row[u][b]);
                    wprod *= wt[u];
                }
            }
            const uint32_t lid = min(h & 0xFFFFFFu, f.n_illum - 1u);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float4 lc = LDS ? s_light[lid * NB + b]
                                      : ld4(f.lcodes + int64_t(lid) * f.ld_l + 4 * (f.block_first + b));
                acc[b] = add4(acc[b], mul4(scale4(lc, wprod), prod[b]));
            }
        }
    }
    // sample mean over the pixel's lanes: xor butterfly inside the segment
    for (int m = 1; m < seg; m <<= 1) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            acc[b].x += shfl_xor(acc[b].x, m);
            acc[b].y += shfl_xor(acc[b].y, m);
            acc[b].z += shfl_xor(acc[b].z, m);
        }
    }
    if (pix_ok && j0 == 0) {
        if constexpr (XYZ) {
            // the same mean the latent image holds, then the decode's dot
            float z[3 * NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                z[3 * b] = acc[b].x * f.inv_spp;
                z[3 * b + 1] = acc[b].y * f.inv_spp;
                z[3 * b + 2] = acc[b].z * f.inv_spp;
            }
            float x, y, w;
            decode_dot<NB>(s_M, z, x, y, w);
            float* o = f.xyz + q * 3;
            stg_f32(o + 0, x);
            stg_f32(o + 1, y);
            stg_f32(o + 2, w);
        } else {
            float* out = f.zimg + q * f.ld_z + 4 * f.block_first;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                st4(out + 4 * b, make_float4(acc[b].x * f.inv_spp, acc[b].y * f.inv_spp,
                                             acc[b].z * f.inv_spp, 0.f));
            }
        }
    }
}

// Dynamic LDS: the light codes (when they fit), then with XYZ the 9NB
// floats of the decoder matrix.
template <int NB, bool FAR, bool XYZ>
__global__ __launch_bounds__(kBlock) void shade_latent_kernel(LatentFrame f, int lights_in_lds) {
    extern __shared__ float4 s_light[];
    float* s_M = reinterpret_cast<float*>(s_light + (lights_in_lds ? f.n_illum * NB : 0u));
    if (lights_in_lds || XYZ) {
        if (lights_in_lds) stage_lights<NB>(f, s_light);
        if constexpr (XYZ)
            for (int e = threadIdx.x; e < 9 * NB; e += kBlock) s_M[e] = f.M[e];
        __syncthreads();
    }
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    const int64_t q0 = wave * f.P.pw;
    if (q0 >= f.P.n_pixels) return;  // whole wave leaves together; no barrier follows
    if (lights_in_lds)
        latent_group<NB, true, FAR, XYZ>(f, q0, f.P.n_pixels, s_light, s_M);
    else
        latent_group<NB, false, FAR, XYZ>(f, q0, f.P.n_pixels, s_light, s_M);
}

// Persistent launch over a tile table: block b takes tiles b, b + grid, ...
// and its waves split each tile's pixel groups.  Light codes are staged per
// tile when they fit in the LDS budget.
// Occupancy floor for the tile kernel, per code width: the frame kernel's
// occupancy less one wave where that fits the registers without spills (wider
// codes keep the compiler's choice).  Without it the persistent loop's longer
// live ranges cost one or two waves per SIMD.
constexpr int tile_waves(int nb) { return nb <= 1 ? 8 : (nb == 2 ? 6 : 1); }

// With XYZ the tiles' pixels are decoded with the decoder matrix M (one
// codec for every frame) into the frames' xyz; their latent images are not
// written.
template <int NB, bool XYZ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(tile_waves(NB)))) void shade_latent_tiles_kernel(const hc_frame* __restrict__ frames,
                                                                    int n_frames,
                                                                    const hc_tile* __restrict__ tiles,
                                                                    const int32_t* __restrict__ n_tiles_dev,
                                                                    int max_tiles, const float* __restrict__ M) {
    extern __shared__ float4 s_light[];
    // M is the same for every lane: narrow codes hold it in scalar registers
    // (loaded before any store, so through the scalar cache), wider ones
    // stage it in LDS (read after the first barrier of the tile loop)
    constexpr bool kRegM = XYZ && NB <= 4;
    float m_reg[kRegM ? 9 * NB : 1];
    __shared__ float s_M[XYZ && !kRegM ? 9 * NB : 1];
    if constexpr (kRegM) {
#pragma unroll
        for (int e = 0; e < 9 * NB; ++e) m_reg[e] = M[e];
    } else if constexpr (XYZ) {
        for (int e = threadIdx.x; e < 9 * NB; e += kBlock) s_M[e] = M[e];
    }
    const float* m_use = kRegM ? m_reg : s_M;
    const int n_tiles = min(*n_tiles_dev, max_tiles);
    const int wave = wave_in_block();
    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        int64_t begin, end;
        const hc_tile tile = tiles[t];
        if (!tile_range(tile, frames, n_frames, begin, end)) continue;  // uniform over the block
        const hc_frame& fr = frames[tile.frame];
        LatentFrame f;
        f.P = make_view(fr.hdr, fr.pix_first, fr.vtx, fr.n_pixels, fr.n_vertices, fr.spp, kWave);
        f.codes = fr.tex;
        f.ld = fr.ld_tex;
        f.n_tex = static_cast<uint32_t>(fr.n_texels);
        f.lcodes = fr.lights;
        f.ld_l = fr.ld_lights;
        f.n_illum = static_cast<uint32_t>(fr.n_illum);
        f.block_first = 0;
        f.zimg = fr.image;
        f.ld_z = fr.ld_image;
        f.inv_spp = 1.0f / static_cast<float>(fr.spp);
        f.M = nullptr;
        f.xyz = fr.xyz;
        const bool lds = size_t(f.n_illum) * NB * sizeof(float4) <= kLightLdsBytes;
        __syncthreads();  // the previous tile's waves are done with s_light
        if (lds) stage_lights<NB>(f, s_light);
        __syncthreads();
        const int64_t groups = (end - begin + f.P.pw - 1) / f.P.pw;
        if (lds) {
            for (int64_t g = wave; g < groups; g += kWavesPerBlock)
                latent_group<NB, true, false, XYZ>(f, begin + g * f.P.pw, end, s_light, m_use);
        } else {
            for (int64_t g = wave; g < groups; g += kWavesPerBlock)
                latent_group<NB, false, false, XYZ>(f, begin + g * f.P.pw, end, s_light, m_use);
        }
    }
}

#define HC_NB_CASES(M) \
    M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)

}  // namespace

namespace {

// One frame launch: block_count code blocks from block_first into zimg, or
// (XYZ) all blocks decoded with M into xyz.
template <bool XYZ>
hc_status launch_frame(const hc_paths& P, const hc_latent_assets& A, int block_first, int block_count,
                       float* zimg, int64_t ld_zimg, const float* M, float* xyz, hipStream_t st,
                       const char* fn) {
    LatentFrame f;
    f.P = make_view(P, kWave);
    f.codes = A.codes;
    f.ld = A.ld;
    f.n_tex = static_cast<uint32_t>(A.n_texels);
    f.lcodes = A.illum_codes;
    f.ld_l = A.ld_illum;
    f.n_illum = static_cast<uint32_t>(A.n_illum);
    f.block_first = block_first;
    f.zimg = zimg;
    f.ld_z = ld_zimg;
    f.inv_spp = 1.0f / static_cast<float>(P.spp);
    f.M = M;
    f.xyz = xyz;
    const size_t lds_need = size_t(A.n_illum) * block_count * sizeof(float4);
    const int lights_in_lds = lds_need <= kLightLdsBytes;
    size_t lds = (lights_in_lds ? lds_need : 0) + (XYZ ? size_t(9 * block_count) * sizeof(float) : 0);
    // A code table past the 256 MB cache is read from HBM at random: there
    // fewer gathers in flight are served faster (measured at 1 GiB: half the
    // vertices in flight per lane and at most four waves per SIMD, 52.9 ->
    // 49.0 ms on the 4K / 64 spp frame).  The wave cap is an LDS reservation
    // of a quarter of the CU's 160 KB per four-wave workgroup (which holds the
    // light table and decoder matrix too).
    const bool far = double(A.n_texels) * double(A.ld) * sizeof(float) > kCacheBytes;
    if (far) lds = std::max<size_t>(lds, kFarLdsBytes);
    const int64_t waves = ceil_div(P.n_pixels, f.P.pw);
    const int64_t blocks = ceil_div(waves, kWavesPerBlock);
    if (blocks > 0x7FFFFFFF) {
        set_error("%s: frame too large for one launch", fn);
        return HC_ESHAPE;
    }
    switch (block_count) {
#define HC_CASE(NB)                                                                                \
    case NB:                                                                                       \
        if (far)                                                                                   \
            hipLaunchKernelGGL((shade_latent_kernel<NB, true, XYZ>), dim3(uint32_t(blocks)), dim3(kBlock), \
                               lds, st, f, lights_in_lds);                                         \
        else                                                                                       \
            hipLaunchKernelGGL((shade_latent_kernel<NB, false, XYZ>), dim3(uint32_t(blocks)), dim3(kBlock), \
                               lds, st, f, lights_in_lds);                                         \
        break;
        HC_NB_CASES(HC_CASE)
#undef HC_CASE
        default:
            set_error("%s: block_count %d unsupported", fn, block_count);
            return HC_EUNSUPPORTED;
    }
    return launch_status(fn);
}

}  // namespace

hc_status launch_shade_latent(const hc_paths& P, const hc_latent_assets& A, int block_first,
                              int block_count, float* zimg, int64_t ld_zimg, hipStream_t st) {
    return launch_frame<false>(P, A, block_first, block_count, zimg, ld_zimg, nullptr, nullptr, st,
                               "hc_shade_latent");
}

hc_status launch_shade_latent_xyz(const hc_paths& P, const hc_latent_assets& A, const float* M, float* xyz,
                                  hipStream_t st) {
    return launch_frame<true>(P, A, 0, int(ceil_div(A.k, 3)), nullptr, 0, M, xyz, st,
                              "hc_shade_latent_xyz");
}

namespace {

template <bool XYZ>
hc_status launch_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles, const int32_t* n_tiles,
                       int max_tiles, int k, const float* M, int grid, hipStream_t st, const char* fn) {
    const int nb = int(ceil_div(k, 3));
    const size_t lds = kLightLdsBytes;
    switch (nb) {
#define HC_CASE(NB)                                                                                  \
    case NB: {                                                                                       \
        const int g = tile_grid(grid, shade_latent_tiles_kernel<NB, XYZ>, kBlock, lds, fn);          \
        if (g <= 0) return HC_EDEVICE;                                                               \
        hipLaunchKernelGGL((shade_latent_tiles_kernel<NB, XYZ>), dim3(g), dim3(kBlock), lds, st,     \
                           frames, n_frames, tiles, n_tiles, max_tiles, M);                          \
        break;                                                                                       \
    }
        HC_NB_CASES(HC_CASE)
#undef HC_CASE
        default:
            set_error("%s: k=%d unsupported", fn, k);
            return HC_EUNSUPPORTED;
    }
    return launch_status(fn);
}

}  // namespace

hc_status launch_shade_latent_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                    const int32_t* n_tiles, int max_tiles, int k, int grid,
                                    hipStream_t st) {
    return launch_tiles<false>(frames, n_frames, tiles, n_tiles, max_tiles, k, nullptr, grid, st,
                               "hc_shade_latent_tiles");
}

hc_status launch_shade_latent_xyz_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                        const int32_t* n_tiles, int max_tiles, int k, const float* M, int grid,
                                        hipStream_t st) {
    return launch_tiles<true>(frames, n_frames, tiles, n_tiles, max_tiles, k, M, grid, st,
                              "hc_shade_latent_xyz_tiles");
}

}  // namespace hc
