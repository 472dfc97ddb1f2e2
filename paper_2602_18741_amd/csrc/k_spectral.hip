// Spectral form: light-path throughput over n wavelength samples, XYZ by the
// colour-matching matrix, per-pixel sample mean by shuffles.  Every index
// read from the records is clamped to its buffer.

#include "shade_common.hpp"

namespace hc {
namespace {
using namespace shade;

// G lanes per path; a lane owns the float4 chunks c = qq*G + sub (qq < Q) of
// the n samples, so one load instruction covers G consecutive chunks of each
// path's texel row: one 128-byte line for G = 8.  (4 lanes per path with two
// chunks each ran slower at n = 31: fewer wavefronts fit per SIMD.)
constexpr int kSpecLanes = 8;
// Pixel groups per wavefront in a frame launch: the per-lane set-up (colour
// weights, chunk offsets, scan constants) is shared by that many groups.
constexpr int kSpecGroupsPerWave = 8;

// Where a path's light spectrum comes from: global memory, or the light
// table staged in LDS when it fits the budget.
enum LightMode { kLightGlobal, kLightLds };

// v plus its value in lane i ^ M (M < 32, inside each 32-lane half):
// ds_swizzle in bit-mask mode (and 0x1F, or 0, xor M), no address register.
template <int M>
__device__ __forceinline__ float xor_add(float v) {
    static_assert(M > 0 && M < 32, "swizzle reaches within 32 lanes");
    constexpr int pattern = (M << 10) | 0x1F;
    return v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), pattern));
}

// v plus its value in the lane whose ds_bpermute byte address is addr.
__device__ __forceinline__ float add_from(float v, int addr) {
    return v + __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// Sums of x, y and z over each aligned group of `span` lanes (a power of two
// <= 64), as xor butterflies in the order 1, 2, 4, ...; every lane of the
// group gets the sums.  The three are interleaved step by step so their
// shuffles overlap.  KNOWN is a lower bound on span fixed at compile time:
// the steps below it need no test.
template <int KNOWN = 1>
__device__ __forceinline__ void xor_sum3(float& x, float& y, float& z, int span) {
#define HC_XOR_STEP(M)                                        \
    if (KNOWN > (M) || span > (M)) {                          \
        x = xor_add<(M)>(x);                                  \
        y = xor_add<(M)>(y);                                  \
        z = xor_add<(M)>(z);                                  \
    }
    HC_XOR_STEP(1)
    HC_XOR_STEP(2)
    HC_XOR_STEP(4)
    HC_XOR_STEP(8)
    HC_XOR_STEP(16)
#undef HC_XOR_STEP
    if (span > 32) {
        const int src = (int(threadIdx.x & (kWave - 1)) ^ 32) << 2;
        x = add_from(x, src);
        y = add_from(y, src);
        z = add_from(z, src);
    }
}

// Segmented prefix sum of path lengths over the slots of pixel segments, with
// the per-lane set-up done once: `seg` slots per segment (a power of two), `G`
// lanes per slot, the lane in slot j0 of its segment.  The steps are unrolled
// (at most log2(64 / G)).
template <int G>
struct SegScan {
    static constexpr int kMaxSteps = 6 - __builtin_ctz(unsigned(G));  // log2(64 / G)
    int src[kMaxSteps];  // ds_bpermute byte address of the lane G << i below
    int last;            // byte address of the segment's last slot
    int steps;           // log2(seg)
    int j0;

    __device__ __forceinline__ SegScan(int lane, int seg, int j0_) : j0(j0_) {
        steps = __builtin_ctz(unsigned(seg));
        // (wrapping below lane 0; such a value is used only outside the segment)
#pragma unroll
        for (int i = 0; i < kMaxSteps; ++i) src[i] = ((lane - (G << i)) & (kWave - 1)) << 2;
        const int seg_lanes = seg * G;
        last = ((lane & ~(seg_lanes - 1)) + seg_lanes - 1) << 2;
    }

    // Exclusive prefix of len over the slots of the segment; total gets the
    // segment's sum.
    __device__ __forceinline__ uint32_t exclusive(uint32_t len, uint32_t& total) const {
        uint32_t incl = len;
#pragma unroll
        for (int i = 0; i < kMaxSteps; ++i) {
            if (i < steps) {
                const uint32_t y = uint32_t(__builtin_amdgcn_ds_bpermute(src[i], int(incl)));
                incl += (j0 >= (1 << i)) ? y : 0u;
            }
        }
        total = uint32_t(__builtin_amdgcn_ds_bpermute(last, int(incl)));
        return incl - len;
    }
};

// A row of ones, as long as the longest spectrum: padding vertex slots read
// their row from here, so the product needs no select per loaded chunk.
struct alignas(16) OnesRow {
    float v[kMaxN];
};
constexpr OnesRow make_ones_row() {
    OnesRow r{};
    for (int i = 0; i < kMaxN; ++i) r.v[i] = 1.f;
    return r;
}
__device__ const OnesRow kOnesRow = make_ones_row();

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

// Occupancy floor of the frame kernel: 7 waves per SIMD for one chunk per
// lane (the compiler's choice is 6 for the global-light variant), 6 for two
// (80 registers); wider rows keep the compiler's choice.  None spills.
constexpr int spec_frame_waves(int q) { return q <= 1 ? 7 : (q == 2 ? 6 : 1); }

constexpr size_t light_lds_bytes(uint32_t n_illum, int nq) { return size_t(n_illum) * nq * sizeof(float4); }

// With two or more chunks per lane the colour-matching weights (3 float4 per
// chunk) would hold 24 or more registers for the whole kernel; they are read
// from an LDS copy instead, staged once per block at the start of the shared
// memory (room for n up to 128), the light table after it.
constexpr bool t_in_lds(int q) { return q >= 2; }
constexpr int kTLdsFloat4 = 3 * (kMaxN / 4);

__device__ __forceinline__ void stage_T(const float* T, int n, int nq, float4* s_T) {
    for (int i = threadIdx.x; i < 3 * nq; i += kBlock) {
        const int ch = i / nq, c = i % nq;
        float w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * c + e;
            w[e] = k < n ? ldg_f32(T + ch * n + k) : 0.f;
        }
        s_T[i] = make_float4(w[0], w[1], w[2], w[3]);
    }
}

// What a lane needs for every path it shades, given only the sample count:
// G lanes per path, the lane owning float4 chunks c = qq * G + sub.
template <int G, int Q>
struct SpecLane {
    float4 Tr[3][Q];     // colour-matching weights of the lane's samples, 0 past n
    bool keep[Q][4];     // the lane's samples below n
    bool chunk_ok[Q];    // chunk below the n samples' chunk count
    uint32_t off[Q];     // float offset of chunk qq in a row
};

template <int G, int Q>
__device__ __forceinline__ SpecLane<G, Q> spec_lane(const float* T, int n, int nq) {
    constexpr bool kWithT = !t_in_lds(Q);
    SpecLane<G, Q> L;
    const int sub = threadIdx.x & (G - 1);
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) {
        const int c = qq * G + sub;
        L.chunk_ok[qq] = c < nq;
        // a lane past the n samples re-reads the last chunk; its sums are
        // never used
        L.off[qq] = 4u * uint32_t(min(c, nq - 1));
        // the products of samples past n are replaced by 0 (not multiplied,
        // so non-finite row padding cannot leak in)
#pragma unroll
        for (int e = 0; e < 4; ++e) L.keep[qq][e] = 4 * c + e < n;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float w[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 4 * c + e;
                const float t = kWithT ? ldg_f32(T + ch * n + min(i, n - 1)) : 0.f;
                w[e] = (i < n) ? t : 0.f;
            }
            L.Tr[ch][qq] = make_float4(w[0], w[1], w[2], w[3]);
        }
    }
    return L;
}

// The calling wave shades the pixel groups g = g_begin, g_begin + g_step, ...
// below g_end; group g is pixels [q_base + g * pw, ...), cut at q_end.  The
// light spectra come from global memory or the table s_light staged for mode
// M.  The lane's scan sources are set up once for all groups.
template <int G, int Q, LightMode M>
__device__ __forceinline__ void spectral_groups(const SpectralFrame& f, const SpecLane<G, Q>& L,
                                                int64_t q_base, int64_t q_end, int64_t g_begin,
                                                int64_t g_end, int64_t g_step, const float4* s_light,
                                                const float4* s_T) {
    const PathView& P = f.P;
    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane & (G - 1);
    const int slot = lane / G;
    const int seg = P.spp_pad;  // slots per pixel segment, a power of two
    const int j0 = slot & (seg - 1);
    const int pix = slot >> __builtin_ctz(unsigned(seg));
    const SegScan<G> scan(lane, seg, j0);
    // byte addresses of the lane's first chunk in texel row 0 and in the row
    // of ones, and of its other chunks relative to the first
    const char* lane_refl = reinterpret_cast<const char*>(f.refl + L.off[0]);
    const char* lane_ones = reinterpret_cast<const char*>(kOnesRow.v + L.off[0]);
    const uint32_t row_bytes = uint32_t(f.ld) * 4u;  // ld < 2^30
    uint32_t dq[Q];
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) dq[qq] = 4u * (L.off[qq] - L.off[0]);

    for (int64_t g = g_begin; g < g_end; g += g_step) {
        const int64_t q = q_base + g * P.pw + pix;
        const bool pix_ok = q < q_end;
        uint32_t next = pix_ok ? ldg_u32(P.pix_first + q) : 0u;
        float ax = 0.f, ay = 0.f, az = 0.f;

        for (int r = 0; r < P.rounds; ++r) {
            const int j = j0 + r * seg;
            const bool live = pix_ok && j < P.spp;
            const uint32_t h = live ? ldg_u32(P.hdr + (q * P.spp + j)) : 0u;
            const uint32_t len = h >> 24;
            uint32_t total;
            const uint32_t first = next + scan.exclusive(len, total);
            next += total;
            if (live) {
                float4 prod[Q];
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) prod[qq] = make_float4(1.f, 1.f, 1.f, 1.f);
                float wprod = 1.f;
                const uint32_t end = (first < P.n_vertices) ? min(first + len, P.n_vertices) : first;
                // U vertices at a time: records, then rows, all in flight
                // before the first multiply; padding slots multiply by 1
                constexpr int U = Q <= 2 ? 4 : 2;
                for (uint32_t jv = first; jv < end; jv += U) {
                    // records first, all U in flight: slots past the path read
                    // the following (in-bounds) records, which the wave fetches
                    // anyway
                    uint2 rec[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) rec[u] = ldg_u2(P.vtx + min(jv + u, P.n_vertices - 1u));
                    // rows are loaded unconditionally (no branch per vertex): a
                    // padding slot reads the row of ones and weight 1.  rp is
                    // the address of the lane's first chunk: one multiply-add
                    // from the lane's base (row bytes < 2^32)
                    const char* rp[U];
                    float wt[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool ok = jv + u < end;
                        const uint32_t tex = min(rec[u].x, f.n_tex - 1u);
                        const char* tp = lane_refl + uint64_t(tex) * row_bytes;
                        rp[u] = ok ? tp : lane_ones;
                        wt[u] = ok ? __uint_as_float(rec[u].y) : 1.f;
                    }
                    float4 row[U][Q];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int qq = 0; qq < Q; ++qq)
                            row[u][qq] = ld4(reinterpret_cast<const float*>(rp[u] + dq[qq]));
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int qq = 0; qq < Q; ++qq) prod[qq] = mul4(prod[qq], row[u][qq]);
                        wprod *= wt[u];
                    }
                }
                const uint32_t lid = min(h & 0xFFFFFFu, f.n_illum - 1u);
                float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) {
                    if (L.chunk_ok[qq]) {
                        const int c = qq * G + sub;
                        const float4 lt = M == kLightLds ? s_light[lid * f.nq + c]
                                                         : ld4(f.illum + int64_t(lid) * f.ld_l + 4 * c);
                        const float4 m = mul4(lt, prod[qq]);
                        const float s0 = L.keep[qq][0] ? m.x : 0.f;
                        const float s1 = L.keep[qq][1] ? m.y : 0.f;
                        const float s2 = L.keep[qq][2] ? m.z : 0.f;
                        const float s3 = L.keep[qq][3] ? m.w : 0.f;
                        float4 tx, ty, tz;
                        if constexpr (t_in_lds(Q)) {
                            tx = s_T[c];
                            ty = s_T[f.nq + c];
                            tz = s_T[2 * f.nq + c];
                        } else {
                            tx = L.Tr[0][qq];
                            ty = L.Tr[1][qq];
                            tz = L.Tr[2][qq];
                        }
                        sx += tx.x * s0 + tx.y * s1 + tx.z * s2 + tx.w * s3;
                        sy += ty.x * s0 + ty.y * s1 + ty.z * s2 + ty.w * s3;
                        sz += tz.x * s0 + tz.y * s1 + tz.z * s2 + tz.w * s3;
                    }
                }
                // the vertex weights multiply the whole spectrum
                ax += wprod * sx;
                ay += wprod * sy;
                az += wprod * sz;
            }
        }
        // reduce over the G sample lanes, then over the pixel's slots
        xor_sum3<G>(ax, ay, az, G * seg);
        if (pix_ok && sub == 0 && j0 == 0) {
            float* out = f.xyz + q * 3;
            stg_f32(out + 0, ax * f.inv_spp);
            stg_f32(out + 1, ay * f.inv_spp);
            stg_f32(out + 2, az * f.inv_spp);
        }
    }
}

template <int G, int Q, LightMode M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(spec_frame_waves(Q)))) void shade_spectral_kernel(SpectralFrame f) {
    extern __shared__ float4 s_mem[];
    float4* s_T = s_mem;
    float4* s_light = s_mem + (t_in_lds(Q) ? kTLdsFloat4 : 0);
    if constexpr (t_in_lds(Q)) stage_T(f.T, f.n, f.nq, s_T);
    if constexpr (M == kLightLds) stage_lights(f, s_light);
    if constexpr (t_in_lds(Q) || M == kLightLds) __syncthreads();
    // each wave takes kSpecGroupsPerWave consecutive pixel groups
    const int64_t wave = int64_t(blockIdx.x) * kWavesPerBlock + wave_in_block();
    const int64_t groups = (f.P.n_pixels + f.P.pw - 1) / f.P.pw;
    const int64_t g0 = wave * kSpecGroupsPerWave;
    if (g0 >= groups) return;
    const int64_t g1 = min(g0 + kSpecGroupsPerWave, groups);
    const SpecLane<G, Q> L = spec_lane<G, Q>(f.T, f.n, f.nq);
    spectral_groups<G, Q, M>(f, L, 0, f.P.n_pixels, g0, g1, 1, s_light, s_T);
}

// Occupancy floor for the tile kernel: 6 waves per SIMD for one chunk per
// lane (80 registers, no spills; the compiler's choice is 5).
constexpr int spec_tile_waves(int q) { return q <= 1 ? 6 : 1; }

// Persistent launch over a tile table (see the latent form).
template <int G, int Q>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(spec_tile_waves(Q)))) void shade_spectral_tiles_kernel(const hc_frame* __restrict__ frames,
                                                                      int n_frames,
                                                                      const hc_tile* __restrict__ tiles,
                                                                      const int32_t* __restrict__ n_tiles_dev,
                                                                      int max_tiles, int n,
                                                                      const float* __restrict__ T) {
    extern __shared__ float4 s_mem[];
    float4* s_T = s_mem;
    float4* s_light = s_mem + (t_in_lds(Q) ? kTLdsFloat4 : 0);
    const int n_tiles = min(*n_tiles_dev, max_tiles);
    const int wave = wave_in_block();
    const SpecLane<G, Q> L = spec_lane<G, Q>(T, n, (n + 3) / 4);
    // read after the first tile's barriers below
    if constexpr (t_in_lds(Q)) stage_T(T, n, (n + 3) / 4, s_T);
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
        const bool lds = light_lds_bytes(f.n_illum, f.nq) <= kLightLdsBytes;
        __syncthreads();
        if (lds) stage_lights(f, s_light);
        __syncthreads();
        const int64_t groups = (end - begin + f.P.pw - 1) / f.P.pw;
        if (lds)
            spectral_groups<G, Q, kLightLds>(f, L, begin, end, wave, groups, kWavesPerBlock, s_light, s_T);
        else
            spectral_groups<G, Q, kLightGlobal>(f, L, begin, end, wave, groups, kWavesPerBlock, s_light, s_T);
    }
}

template <int G, int Q>
hc_status launch_spectral_gq(const SpectralFrame& f, int64_t blocks, hipStream_t st) {
    // the light table in LDS if it fits the budget
    const dim3 grid(static_cast<uint32_t>(blocks)), block(kBlock);
    const size_t lights = light_lds_bytes(f.n_illum, f.nq);
    const size_t t_bytes = t_in_lds(Q) ? kTLdsFloat4 * sizeof(float4) : 0;
    if (lights <= kLightLdsBytes)
        hipLaunchKernelGGL((shade_spectral_kernel<G, Q, kLightLds>), grid, block, t_bytes + lights, st, f);
    else
        hipLaunchKernelGGL((shade_spectral_kernel<G, Q, kLightGlobal>), grid, block, t_bytes, st, f);
    return launch_status("hc_shade_spectral");
}

template <int G, int Q>
hc_status launch_spectral_tiles_gq(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                   const int32_t* n_tiles, int max_tiles, int n, const float* T, int grid,
                                   hipStream_t st) {
    const size_t lds = (t_in_lds(Q) ? kTLdsFloat4 * sizeof(float4) : 0) + kLightLdsBytes;
    const int g = tile_grid(grid, shade_spectral_tiles_kernel<G, Q>, kBlock, lds, "hc_shade_spectral_tiles");
    if (g <= 0) return HC_EDEVICE;
    hipLaunchKernelGGL((shade_spectral_tiles_kernel<G, Q>), dim3(g), dim3(kBlock), lds, st, frames, n_frames,
                       tiles, n_tiles, max_tiles, n, T);
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
    const int64_t waves = ceil_div(ceil_div(P.n_pixels, f.P.pw), kSpecGroupsPerWave);
    const int64_t blocks = ceil_div(waves, kWavesPerBlock);
    if (blocks > 0x7FFFFFFF) {
        set_error("hc_shade_spectral: frame too large for one launch");
        return HC_ESHAPE;
    }
    switch (ceil_div(f.nq, kSpecLanes)) {
        case 1: return launch_spectral_gq<kSpecLanes, 1>(f, blocks, st);
        case 2: return launch_spectral_gq<kSpecLanes, 2>(f, blocks, st);
        case 3: return launch_spectral_gq<kSpecLanes, 3>(f, blocks, st);
        case 4: return launch_spectral_gq<kSpecLanes, 4>(f, blocks, st);
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
