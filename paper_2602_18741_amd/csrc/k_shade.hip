// Light-path shading in spectral form (n samples) and latent form (k = 3B code
// channels), with the per-pixel sample mean done by wavefront shuffles.
//
// Work mapping (one 64-lane wavefront = one unit of work):
//   latent   : one lane per path.  Lanes of a pixel are contiguous (spp padded
//              to a power of two up to 64; larger spp loops over rounds of 64
//              paths).  A lane gathers ceil-blocks of 16 bytes per vertex.
//   spectral : eight lanes per path, each owning float4 chunks c = 8*qq + sub
//              of the n samples, so the eight lanes of a path read one 128-byte
//              line of the texel row per instruction.  Eight paths per wave.
// Path records stream in pixel order; the first-vertex offset of each path is
// a segmented prefix sum of path lengths done with shuffles.  Light tables
// that fit are staged in LDS.  Every index read from the records is clamped
// to its buffer, so malformed records cannot move a read outside the inputs.

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr size_t kLightLdsBytes = 16384;

struct PathView {
    const uint32_t* hdr;
    const uint32_t* pix_first;
    const uint2* vtx;
    int64_t n_pixels;
    uint32_t n_vertices;
    int spp;
    int spp_pad;  // slots per pixel inside one round (power of two)
    int pw;       // pixels per wave
    int rounds;   // rounds of paths per pixel
};

// Paths-per-wave layout shared by both forms: `slots` path slots per wave.
PathView make_view(const hc_paths& P, int slots) {
    PathView v;
    v.hdr = P.hdr;
    v.pix_first = P.pix_first;
    v.vtx = reinterpret_cast<const uint2*>(P.vtx);
    v.n_pixels = P.n_pixels;
    v.n_vertices = static_cast<uint32_t>(P.n_vertices);
    v.spp = P.spp;
    if (P.spp <= slots) {
        int pad = 1;
        while (pad < P.spp) pad <<= 1;
        v.spp_pad = pad;
        v.pw = slots / pad;
        v.rounds = 1;
    } else {
        v.spp_pad = slots;
        v.pw = 1;
        v.rounds = static_cast<int>(ceil_div(P.spp, slots));
    }
    return v;
}

// Exclusive prefix of `len` over the slots of one pixel segment of `seg`
// slots, `lanes_per_slot` lanes apart.  `j0` is the slot's index inside its
// segment.  Returns the exclusive prefix; `total` gets the segment's sum.
__device__ __forceinline__ uint32_t segment_scan(uint32_t len, int j0, int seg, int lanes_per_slot,
                                                 uint32_t& total) {
    uint32_t incl = len;
    for (int d = 1; d < seg; d <<= 1) {
        uint32_t y = shfl_up_u32(incl, d * lanes_per_slot);
        if (j0 >= d) incl += y;
    }
    // the last slot of the segment holds the segment total
    const int lane = threadIdx.x & (kWave - 1);
    const int seg_lanes = seg * lanes_per_slot;
    const int last = (lane / seg_lanes) * seg_lanes + seg_lanes - 1;
    total = shfl_u32(incl, last);
    return incl - len;
}

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
            for (uint32_t jv = first; jv < end; ++jv) {
                const uint2 rec = P.vtx[jv];
                const uint32_t t = min(rec.x, a.n_tex - 1u);
                const float* row = a.codes + int64_t(t) * a.ld + 4 * a.block_first;
#pragma unroll
                for (int b = 0; b < NB; ++b) prod[b] = mul4(prod[b], ld4(row + 4 * b));
                wprod *= __uint_as_float(rec.y);
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

// ------------------------------------------------------------------ spectral form

constexpr int kSpecLanes = 8;  // lanes per path
constexpr int kSpecSlots = kWave / kSpecLanes;

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

template <int Q>
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
    const int sub = lane & (kSpecLanes - 1);
    const int slot = lane / kSpecLanes;
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t q0 = wave * P.pw;
    if (q0 >= P.n_pixels) return;

    // colour-matching weights of this lane's samples; zero past n
    float4 Tr[3][Q];
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) {
        const int c = qq * kSpecLanes + sub;
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
        const uint32_t first = next + segment_scan(len, j0, seg, kSpecLanes, total);
        next += total;
        if (live) {
            float4 prod[Q];
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) prod[qq] = make_float4(1.f, 1.f, 1.f, 1.f);
            float wprod = 1.f;
            const uint32_t end = (first < P.n_vertices) ? min(first + len, P.n_vertices) : first;
            for (uint32_t jv = first; jv < end; ++jv) {
                const uint2 rec = P.vtx[jv];
                const uint32_t t = min(rec.x, a.n_tex - 1u);
                const float* row = a.refl + int64_t(t) * a.ld;
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) {
                    const int c = qq * kSpecLanes + sub;
                    if (c < a.nq) prod[qq] = mul4(prod[qq], ld4(row + 4 * c));
                }
                wprod *= __uint_as_float(rec.y);
            }
            const uint32_t lid = min(h & 0xFFFFFFu, a.n_illum - 1u);
#pragma unroll
            for (int qq = 0; qq < Q; ++qq) {
                const int c = qq * kSpecLanes + sub;
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
    // reduce over the 8 sample lanes, then over the pixel's slots
    const int span = kSpecLanes * seg;
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

// ------------------------------------------------------------------ record check

struct CheckArgs {
    const uint32_t* hdr;
    const uint32_t* pix_first;
    const uint2* vtx;
    int64_t n_pixels;
    int spp;
    uint64_t n_vertices;
    uint64_t n_tex;
    uint32_t n_illum;
    unsigned long long* counts;
};

__global__ void zero_counts_kernel(unsigned long long* c) {
    if (threadIdx.x < 3) c[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kBlock) void check_paths_kernel(CheckArgs a) {
    const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    unsigned long long bad_light = 0, bad_tex = 0, bad_range = 0;
    if (q < a.n_pixels) {
        uint64_t len_sum = 0;
        for (int j = 0; j < a.spp; ++j) {
            const uint32_t h = a.hdr[q * a.spp + j];
            len_sum += h >> 24;
            bad_light += ((h & 0xFFFFFFu) >= a.n_illum) ? 1 : 0;
        }
        const uint64_t first = a.pix_first[q];
        if (first + len_sum > a.n_vertices) {
            bad_range = 1;
        } else {
            for (uint64_t jv = first; jv < first + len_sum; ++jv)
                bad_tex += (a.vtx[jv].x >= a.n_tex) ? 1 : 0;
        }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        bad_light += __shfl_xor(bad_light, m, kWave);
        bad_tex += __shfl_xor(bad_tex, m, kWave);
        bad_range += __shfl_xor(bad_range, m, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (bad_light) atomicAdd(&a.counts[0], bad_light);
        if (bad_tex) atomicAdd(&a.counts[1], bad_tex);
        if (bad_range) atomicAdd(&a.counts[2], bad_range);
    }
}

template <int NB>
hc_status launch_latent_nb(const LatentArgs& a, int64_t blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(shade_latent_kernel<NB>, dim3(uint32_t(blocks)), dim3(kBlock), lds, st, a);
    return launch_status("hc_shade_latent");
}

template <int Q>
hc_status launch_spectral_q(const SpectralArgs& a, int64_t blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(shade_spectral_kernel<Q>, dim3(uint32_t(blocks)), dim3(kBlock), lds, st, a);
    return launch_status("hc_shade_spectral");
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

hc_status launch_shade_spectral(const hc_paths& P, const hc_spectral_assets& A, const float* T,
                                float* xyz, hipStream_t st) {
    SpectralArgs a;
    a.P = make_view(P, kSpecSlots);
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
        case 1: return launch_spectral_q<1>(a, blocks, lds, st);
        case 2: return launch_spectral_q<2>(a, blocks, lds, st);
        case 3: return launch_spectral_q<3>(a, blocks, lds, st);
        case 4: return launch_spectral_q<4>(a, blocks, lds, st);
        default:
            set_error("hc_shade_spectral: n=%d unsupported", A.n);
            return HC_EUNSUPPORTED;
    }
}

hc_status launch_check_paths(const hc_paths& P, int64_t n_texels, int32_t n_illum, uint64_t* counts,
                             hipStream_t st) {
    CheckArgs a;
    a.hdr = P.hdr;
    a.pix_first = P.pix_first;
    a.vtx = reinterpret_cast<const uint2*>(P.vtx);
    a.n_pixels = P.n_pixels;
    a.spp = P.spp;
    a.n_vertices = static_cast<uint64_t>(P.n_vertices);
    a.n_tex = static_cast<uint64_t>(n_texels);
    a.n_illum = static_cast<uint32_t>(n_illum);
    a.counts = reinterpret_cast<unsigned long long*>(counts);
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(kWave), 0, st, a.counts);
    hc_status s = launch_status("hc_check_paths");
    if (s != HC_OK || P.n_pixels == 0) return s;
    const int64_t blocks = ceil_div(P.n_pixels, kBlock);
    hipLaunchKernelGGL(check_paths_kernel, dim3(uint32_t(blocks)), dim3(kBlock), 0, st, a);
    return launch_status("hc_check_paths");
}

}  // namespace hc
