// Latent form: light-path throughput in code space.  One lane per path; a
// pixel's paths are contiguous lanes (spp padded to a power of two up to 64,
// larger spp loops over rounds of 64 paths).  Per vertex a lane gathers the
// 16-byte blocks of the texel's code (blocked RGBx layout) and multiplies
// them into its product, block by block (the blockwise Hadamard product);
// the light code comes from LDS; the per-pixel sample mean is an xor
// butterfly across the pixel's lanes.  Every index read from the records is
// clamped to its buffer.

#include "shade_common.hpp"

namespace hc {
namespace {
using namespace shade;

// ------------------------------------------------------------------ latent form

struct LatentArgs {
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
    int lights_in_lds;
};

template <int NB>
__global__ __launch_bounds__(kBlock) void shade_latent_kernel(LatentArgs a) {
#pragma clang fp contract(off)
    extern __shared__ float4 s_light[];
    if (a.lights_in_lds) {
        for (uint32_t i = threadIdx.x; i < a.n_illum * NB; i += kBlock) {
            const uint32_t l = i / NB, b = i % NB;
            s_light[i] = ld4(a.lcodes + int64_t(l) * a.ld_l + 4 * (a.block_first + int(b)));
        }
        __syncthreads();
    }
    const PathView& P = a.P;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t q0 = wave * P.pw;
    if (q0 >= P.n_pixels) return;  // whole wave leaves together; no barrier follows

    const int seg = P.spp_pad;                // lanes per pixel segment
    const int j0 = lane % seg;
    const int64_t q = q0 + lane / seg;
    const bool pix_ok = q < P.n_pixels;
    uint32_t next = pix_ok ? P.pix_first[q] : 0u;

    float4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = make_float4(0.f, 0.f, 0.f, 0.f);

    for (int r = 0; r < P.rounds; ++r) {
        const int j = j0 + r * seg;
        const bool live = pix_ok && j < P.spp;
        const uint32_t h = live ? P.hdr[q * P.spp + j] : 0u;
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
            constexpr int U = NB <= 4 ? 4 : (NB <= 8 ? 2 : 1);
            for (uint32_t jv = first; jv < end; jv += U) {
                uint2 rec[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    rec[u] = (jv + u < end) ? P.vtx[jv + u] : make_uint2(0u, 0x3F800000u);
                float4 row[U][NB];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t t = min(rec[u].x, a.n_tex - 1u);
                    const float* rp = a.codes + int64_t(t) * a.ld + 4 * a.block_first;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        row[u][b] = (jv + u < end) ? ld4(rp + 4 * b) : make_float4(1.f, 1.f, 1.f, 1.f);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) prod[b] = mul4(prod[b], row[u][b]);
                    wprod *= __uint_as_float(rec[u].y);
                }
            }
            const uint32_t lid = min(h & 0xFFFFFFu, a.n_illum - 1u);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float4 lc = a.lights_in_lds
                                      ? s_light[lid * NB + b]
                                      : ld4(a.lcodes + int64_t(lid) * a.ld_l + 4 * (a.block_first + b));
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
        float* out = a.zimg + q * a.ld_z + 4 * a.block_first;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            st4(out + 4 * b, make_float4(acc[b].x * a.inv_spp, acc[b].y * a.inv_spp,
                                         acc[b].z * a.inv_spp, 0.f));
        }
    }
}

template <int NB>
hc_status launch_latent_nb(const LatentArgs& a, int64_t blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(shade_latent_kernel<NB>, dim3(uint32_t(blocks)), dim3(kBlock), lds, st, a);
    return launch_status("hc_shade_latent");
}

}  // namespace

hc_status launch_shade_latent(const hc_paths& P, const hc_latent_assets& A, int block_first,
                              int block_count, float* zimg, int64_t ld_zimg, hipStream_t st) {
    LatentArgs a;
    a.P = make_view(P, kWave);
    a.codes = A.codes;
    a.ld = A.ld;
    a.n_tex = static_cast<uint32_t>(A.n_texels);
    a.lcodes = A.illum_codes;
    a.ld_l = A.ld_illum;
    a.n_illum = static_cast<uint32_t>(A.n_illum);
    a.block_first = block_first;
    a.zimg = zimg;
    a.ld_z = ld_zimg;
    a.inv_spp = 1.0f / static_cast<float>(P.spp);
    const size_t lds_need = size_t(A.n_illum) * block_count * sizeof(float4);
    a.lights_in_lds = lds_need <= kLightLdsBytes;
    const size_t lds = a.lights_in_lds ? lds_need : 0;
    const int64_t waves = ceil_div(P.n_pixels, a.P.pw);
    const int64_t blocks = ceil_div(waves, kWavesPerBlock);
    if (blocks > 0x7FFFFFFF) {
        set_error("hc_shade_latent: frame too large for one launch");
        return HC_ESHAPE;
    }
    switch (block_count) {
        case 1: return launch_latent_nb<1>(a, blocks, lds, st);
        case 2: return launch_latent_nb<2>(a, blocks, lds, st);
        case 3: return launch_latent_nb<3>(a, blocks, lds, st);
        case 4: return launch_latent_nb<4>(a, blocks, lds, st);
        case 5: return launch_latent_nb<5>(a, blocks, lds, st);
        case 6: return launch_latent_nb<6>(a, blocks, lds, st);
        case 7: return launch_latent_nb<7>(a, blocks, lds, st);
        case 8: return launch_latent_nb<8>(a, blocks, lds, st);
        case 9: return launch_latent_nb<9>(a, blocks, lds, st);
        case 10: return launch_latent_nb<10>(a, blocks, lds, st);
        case 11: return launch_latent_nb<11>(a, blocks, lds, st);
        case 12: return launch_latent_nb<12>(a, blocks, lds, st);
        case 13: return launch_latent_nb<13>(a, blocks, lds, st);
        case 14: return launch_latent_nb<14>(a, blocks, lds, st);
        case 15: return launch_latent_nb<15>(a, blocks, lds, st);
        case 16: return launch_latent_nb<16>(a, blocks, lds, st);
        default:
            set_error("hc_shade_latent: block_count %d unsupported", block_count);
            return HC_EUNSUPPORTED;
    }
}

}  // namespace hc
