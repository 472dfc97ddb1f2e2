// Pieces shared by the two shading forms: the path-record view, the
// pixel-to-wave mapping and the segmented prefix sum of path lengths.
#pragma once

#include "hc_internal.hpp"

namespace hc {
namespace shade {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr size_t kLightLdsBytes = 16384;
constexpr double kCacheBytes = 256.0 * 1024 * 1024;   // MI355X Infinity Cache (MALL)
constexpr size_t kFarLdsBytes = 40960;                 // a quarter of a CU's LDS

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

// Paths-per-wave layout: `slots` path slots per wave.  Up to `slots`
// samples per pixel, a pixel takes spp rounded up to a power of two slots and
// a wave holds slots / that many pixels; more samples loop over rounds.
__host__ __device__ inline PathView make_view(const uint32_t* hdr, const uint32_t* pix_first,
                                              const uint32_t* vtx, int64_t n_pixels,
                                              int64_t n_vertices, int spp, int slots) {
    PathView v;
    v.hdr = hdr;
    v.pix_first = pix_first;
    v.vtx = reinterpret_cast<const uint2*>(vtx);
    v.n_pixels = n_pixels;
    v.n_vertices = static_cast<uint32_t>(n_vertices);
    v.spp = spp;
    if (spp <= slots) {
        int pad = 1;
        while (pad < spp) pad <<= 1;
        v.spp_pad = pad;
        v.pw = slots / pad;
        v.rounds = 1;
    } else {
        v.spp_pad = slots;
        v.pw = 1;
        v.rounds = (spp + slots - 1) / slots;
    }
    return v;
}

inline PathView make_view(const hc_paths& P, int slots) {
    return make_view(P.hdr, P.pix_first, P.vtx, P.n_pixels, P.n_vertices, P.spp, slots);
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

// The wavefront's index in its workgroup, as a value the compiler knows to be
// uniform across the wavefront (kept in a scalar register, so everything
// derived from it - pixel ranges, loop bounds - stays scalar too).
__device__ __forceinline__ int wave_in_block() {
    return __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
}

// Tile-table launches: a fixed grid walks the tiles; a tile's entries are
// checked against the table sizes so a bad entry is skipped, not followed.
__device__ __forceinline__ bool tile_range(const hc_tile& t, const hc_frame* frames, int n_frames,
                                           int64_t& begin, int64_t& end) {
    if (t.frame < 0 || t.frame >= n_frames) return false;
    const int64_t np = frames[t.frame].n_pixels;
    begin = t.begin < 0 ? 0 : t.begin;
    end = t.end > np ? np : t.end;
    return begin < end;
}

}  // namespace shade
}  // namespace hc
