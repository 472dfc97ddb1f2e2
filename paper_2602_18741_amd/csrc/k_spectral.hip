// Spectral form: light-path throughput over n wavelength samples, XYZ by the
// colour-matching matrix, per-pixel sample mean by shuffles.  Every index
// read from the records is clamped to its buffer.

#include "shade_common.hpp"

namespace hc {
namespace {
using namespace shade;

// G lanes per path, G dividing 64; a lane owns the float4 chunks
// c = qq*G + sub (qq < Q) of the n samples, so one load instruction covers G
// consecutive chunks of each path's texel row (one 128-byte line for G = 8).
#ifndef HC_SPECTRAL_LANES
#define HC_SPECTRAL_LANES 8
#endif
constexpr int kSpecLanes = HC_SPECTRAL_LANES;

struct SpectralArgs {
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
    int lights_in_lds;
};

template <int G, int Q>
__global__ __launch_bounds__(kBlock) void shade_spectral_kernel(SpectralArgs a) {
    extern __shared__ float4 s_light[];
    if (a.lights_in_lds) {
        for (uint32_t i = threadIdx.x; i < a.n_illum * uint32_t(a.nq); i += kBlock) {
            const uint32_t l = i / a.nq, c = i % a.nq;
            s_light[i] = ld4(a.illum + int64_t(l) * a.ld_l + 4 * c);
        }
        __syncthreads();
    }
    const PathView& P = a.P;
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane & (G - 1);
    const int slot = lane / G;
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t q0 = wave * P.pw;
    if (q0 >= P.n_pixels) return;

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
                w[e] = (i < a.n) ? a.T[ch * a.n + i] : 0.f;
            }
            Tr[ch][qq] = make_float4(w[0], w[1], w[2], w[3]);
        }
    }

    const int seg = P.spp_pad;  // slots per pixel segment
    const int j0 = slot % seg;
    const int64_t q = q0 + slot / seg;
    const bool pix_ok = q < P.n_pixels;
    uint32_t next = pix_ok ? P.pix_first[q] : 0u;
    float ax = 0.f, ay = 0.f, az = 0.f;

    for (int r = 0; r < P.rounds; ++r) {
        const int j = j0 + r * seg;
        const bool live = pix_ok && j < P.spp;
        const uint32_t h = live ? P.hdr[q * P.spp + j] : 0u;
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
                uint2 rec[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    rec[u] = (jv + u < end) ? P.vtx[jv + u] : make_uint2(0u, 0x3F800000u);
                float4 row[U][Q];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t t = min(rec[u].x, a.n_tex - 1u);
                    const float* rp = a.refl + int64_t(t) * a.ld;
#pragma unroll
                    for (int qq = 0; qq < Q; ++qq) {
                        const int c = qq * G + sub;
                        row[u][qq] = (jv + u < end && c < a.nq) ? ld4(rp + 4 * c)
                                                                 : make_float4(1.f, 1.f, 1.f, 1.f);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int qq = 0; qq < Q; ++qq) prod[qq] = mul4(prod[qq], row[u][qq]);
                    wprod *= __uint_as_float(rec[u].y);
                }
            }
            const uint32_t lid = min(h & 0xFFFFFFu, a.n_illum - 1u);
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) {
                const int c = qq * G + sub;
                if (c < a.nq) {
                    const float4 lt = a.lights_in_lds ? s_light[lid * a.nq + c]
                                                      : ld4(a.illum + int64_t(lid) * a.ld_l + 4 * c);
                    float4 s = mul4(scale4(lt, wprod), prod[qq]);
                    // samples past n carry no colour weight; drop them so
                    // non-finite row padding cannot leak in
                    if (4 * c + 3 >= a.n) {
                        if (4 * c + 0 >= a.n) s.x = 0.f;
                        if (4 * c + 1 >= a.n) s.y = 0.f;
                        if (4 * c + 2 >= a.n) s.z = 0.f;
                        if (4 * c + 3 >= a.n) s.w = 0.f;
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
        float* out = a.xyz + q * 3;
        out[0] = ax * a.inv_spp;
        out[1] = ay * a.inv_spp;
        out[2] = az * a.inv_spp;
    }
}

template <int G, int Q>
hc_status launch_spectral_gq(const SpectralArgs& a, int64_t blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((shade_spectral_kernel<G, Q>), dim3(uint32_t(blocks)), dim3(kBlock), lds, st, a);
    return launch_status("hc_shade_spectral");
}

}  // namespace

hc_status launch_shade_spectral(const hc_paths& P, const hc_spectral_assets& A, const float* T,
                                float* xyz, hipStream_t st) {
    SpectralArgs a;
    a.P = make_view(P, kWave / kSpecLanes);
    a.refl = A.refl;
    a.ld = A.ld;
    a.n_tex = static_cast<uint32_t>(A.n_texels);
    a.illum = A.illum;
    a.ld_l = A.ld_illum;
    a.n_illum = static_cast<uint32_t>(A.n_illum);
    a.n = A.n;
    a.nq = static_cast<int>(ceil_div(A.n, 4));
    a.T = T;
    a.xyz = xyz;
    a.inv_spp = 1.0f / static_cast<float>(P.spp);
    const size_t lds_need = size_t(A.n_illum) * a.nq * sizeof(float4);
    a.lights_in_lds = lds_need <= kLightLdsBytes;
    const size_t lds = a.lights_in_lds ? lds_need : 0;
    const int64_t waves = ceil_div(P.n_pixels, a.P.pw);
    const int64_t blocks = ceil_div(waves, kWavesPerBlock);
    if (blocks > 0x7FFFFFFF) {
        set_error("hc_shade_spectral: frame too large for one launch");
        return HC_ESHAPE;
    }
    const int q = static_cast<int>(ceil_div(a.nq, kSpecLanes));
    switch (q) {
        case 1: return launch_spectral_gq<kSpecLanes, 1>(a, blocks, lds, st);
        case 2: return launch_spectral_gq<kSpecLanes, 2>(a, blocks, lds, st);
        case 3: return launch_spectral_gq<kSpecLanes, 3>(a, blocks, lds, st);
        case 4: return launch_spectral_gq<kSpecLanes, 4>(a, blocks, lds, st);
        case 5: return launch_spectral_gq<kSpecLanes, 5>(a, blocks, lds, st);
        case 6: return launch_spectral_gq<kSpecLanes, 6>(a, blocks, lds, st);
        case 7: return launch_spectral_gq<kSpecLanes, 7>(a, blocks, lds, st);
        case 8: return launch_spectral_gq<kSpecLanes, 8>(a, blocks, lds, st);
        default:
            set_error("hc_shade_spectral: n=%d unsupported", A.n);
            return HC_EUNSUPPORTED;
    }
}

}  // namespace hc
