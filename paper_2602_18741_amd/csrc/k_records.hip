// Validation of light-path records: counts of out-of-range light ids,
// texel ids and pixel record ranges.

#include "shade_common.hpp"

namespace hc {
namespace {
using namespace shade;

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

}  // namespace

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
