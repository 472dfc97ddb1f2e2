// Pieces shared by the two shading forms: the path-record view, the
// pixel-to-wave mapping and the segmented prefix sum of path lengths.
#pragma once

#include "hc_internal.hpp"

namespace hc {
namespace shade {

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
inline PathView make_view(const hc_paths& P, int slots) {
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


}  // namespace shade
}  // namespace hc
