// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "../../include/hc.h"

namespace hc {

// ---------------------------------------------------------------- errors

void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

// Checks the launch that was just enqueued.
hc_status launch_status(const char* what);

// Grid of a persistent tile-table launch that the caller left to the library
// (grid <= 0): twice the number of workgroups of `kernel` (`threads` threads,
// `lds` bytes of dynamic LDS) the current device holds at once, so the grid
// is a whole number of rounds of resident workgroups and none of a partly
// filled second round finishes after the rest.  A grid > 0 is kept.  Returns
// 0 (with the error set) if the device cannot be queried.
template <typename K>
int tile_grid(int grid, K kernel, int threads, size_t lds, const char* what) {
    if (grid > 0) return grid;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
        cus <= 0 || per_cu <= 0) {
        set_error("%s: occupancy query failed", what);
        return 0;
    }
    return 2 * cus * per_cu;
}

// Workgroups of `kernel` (with `threads` threads and `lds` bytes of dynamic
// LDS) the current device holds at once, for persistent launches; the
// occupancy query is made once per device, kernel and LDS size.  Returns 0
// (with the error set) if the device cannot be queried.
template <typename K>
int resident_grid(K kernel, int threads, size_t lds, const char* what) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("%s: no current device", what);
        return 0;
    }
    const auto key = std::make_tuple(dev, reinterpret_cast<const void*>(kernel), lds);
    {
        std::lock_guard<std::mutex> g(mu);
        const auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
        cus <= 0 || per_cu <= 0) {
        set_error("%s: occupancy query failed", what);
        return 0;
    }
    std::lock_guard<std::mutex> g(mu);
    cache[key] = cus * per_cu;
    return cus * per_cu;
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
inline bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kWave = 64;
constexpr int kMaxN = 128;
constexpr int kMaxK = 48;
constexpr int kMaxBlocks = kMaxK / 3;  // 16 float4 slots per latent row

// ---------------------------------------------------------------- device helpers

// Device-memory accesses through the global address space: pointers read
// from device tables would otherwise be generic and compile to flat
// instructions.  Every buffer the library touches is global memory.
#define HC_GLOBAL __attribute__((address_space(1)))
typedef float hc_v4f __attribute__((ext_vector_type(4)));
typedef unsigned int hc_v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float4 ld4(const float* p) {
    const hc_v4f v = *(const HC_GLOBAL hc_v4f*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(float* p, float4 v) {
    const hc_v4f t = {v.x, v.y, v.z, v.w};
    *(HC_GLOBAL hc_v4f*)p = t;
}
__device__ __forceinline__ uint2 ldg_u2(const uint2* p) {
    const hc_v2u v = *(const HC_GLOBAL hc_v2u*)p;
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint32_t ldg_u32(const uint32_t* p) {
    return *(const HC_GLOBAL uint32_t*)p;
}
__device__ __forceinline__ float ldg_f32(const float* p) { return *(const HC_GLOBAL float*)p; }
__device__ __forceinline__ void stg_f32(float* p, float v) { *(HC_GLOBAL float*)p = v; }
__device__ __forceinline__ float4 mul4(float4 a, float4 b) {
    return make_float4(a.x * b.x, a.y * b.y, a.z * b.z, a.w * b.w);
}
__device__ __forceinline__ float4 scale4(float4 a, float s) {
    return make_float4(a.x * s, a.y * s, a.z * s, a.w * s);
}
__device__ __forceinline__ float4 add4(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// Lane-level shuffles inside one 64-wide wavefront.
__device__ __forceinline__ float shfl_xor(float v, int mask) { return __shfl_xor(v, mask, kWave); }
__device__ __forceinline__ uint32_t shfl_up_u32(uint32_t v, int d) {
    return static_cast<uint32_t>(__shfl_up(static_cast<int>(v), d, kWave));
}
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int lane) {
    return static_cast<uint32_t>(__shfl(static_cast<int>(v), lane, kWave));
}

// ---------------------------------------------------------------- launchers (per TU)

hc_status launch_encode(const float* E, int k, int n, const float* S, int64_t m, int64_t ld_s,
                        float* Z, int64_t ld_z, hipStream_t st);
hc_status launch_decode(const float* D, int n, int k, const float* T, const float* zimg,
                        int64_t n_pixels, int64_t ld_zimg, float* xyz, float* spectra,
                        int64_t ld_spectra, hipStream_t st);
hc_status launch_shade_spectral(const hc_paths& P, const hc_spectral_assets& A, const float* T,
                                float* xyz, hipStream_t st);
hc_status launch_shade_latent(const hc_paths& P, const hc_latent_assets& A, int block_first,
                              int block_count, float* zimg, int64_t ld_zimg, hipStream_t st);
hc_status launch_shade_latent_xyz(const hc_paths& P, const hc_latent_assets& A, const float* M, float* xyz,
                                  hipStream_t st);
hc_status launch_decode_matrix(const float* D, int n, int k, const float* T, float* M, hipStream_t st);
hc_status launch_shade_latent_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                    const int32_t* n_tiles, int max_tiles, int k, int grid,
                                    hipStream_t st);
hc_status launch_shade_latent_xyz_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                        const int32_t* n_tiles, int max_tiles, int k, const float* M, int grid,
                                        hipStream_t st);
hc_status launch_shade_spectral_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                                      const int32_t* n_tiles, int max_tiles, int n, const float* T,
                                      int grid, hipStream_t st);
hc_status launch_decode_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                              const int32_t* n_tiles, int max_tiles, const float* D, int n, int k,
                              const float* T, int grid, hipStream_t st);
hc_status launch_encode_jobs(const hc_encode_job* jobs, const int32_t* n_jobs, int max_jobs,
                             const float* E, int k, int n, int grid, hipStream_t st);
hc_status launch_check_paths(const hc_paths& P, int64_t n_texels, int32_t n_illum,
                             uint64_t* counts, hipStream_t st);
hc_status launch_codec_step(const hc_codec_args& a);
size_t codec_static_need(const hc_codec_args& a);
hc_status launch_codec_step_static(const hc_codec_args& a);
int64_t upsample_param_count(int k);
size_t upsample_train_workspace_size(int k, int64_t N);
hc_status launch_upsample_train(const hc_upsample_train_args& a);
hc_status launch_upsample(const hc_mlp& net, int precision, const float* rgb, int64_t m,
                          int64_t ld_rgb, float* Z, int64_t ld_z, hipStream_t st);
size_t codec_workspace_size(int k, int n, int64_t N);
hc_status launch_codec_weights(const void* we, const void* wd, int k, int n, int dtype,
                               double beta, float* E, float* D, hipStream_t st);
size_t gen_workspace_size(int64_t n_pixels);
hc_status launch_gen_headers(const hc_path_gen& g, uint32_t* hdr, uint32_t* pix_first,
                             uint64_t* n_vertices, void* ws, size_t ws_bytes, hipStream_t st);
hc_status launch_gen_vertices(const hc_path_gen& g, const uint32_t* pix_first, uint32_t* vtx,
                              int64_t n_vertices, hipStream_t st);
hc_status launch_gen_indices(uint64_t seed, uint64_t ctr0, const int64_t* scale, int64_t count,
                             int64_t n, uint32_t* out, hipStream_t st);
hc_status launch_gather_probe(const uint2* vtx, uint32_t nv, const float* table, uint32_t n_rows,
                              uint32_t ld, int row_floats, int unroll, int lanes_per_row, float* out,
                              int grid, hipStream_t st);
hc_status launch_stream_probe(const float* src, float* dst, uint64_t n16, int mode, int grid, hipStream_t st);

}  // namespace hc
