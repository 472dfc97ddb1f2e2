// Counter-based random numbers: SplitMix64's output function (Steele, Lea and
// Flood, OOPSLA 2014) applied to key + (counter + 1) * 0x9E3779B97F4A7C15,
// with key = mix64(mix64(seed) + stream).  Used by the synthetic path-record
// generator and by the random pair indices of codec fitting (hc_gen_indices
// and the pair draw of hc_codec_step), so any value is reproducible on its own.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hc {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kIndexStream = 3;  // stream of the random pair indices

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(mix64(seed) + stream);
}
__device__ __forceinline__ uint64_t rand64(uint64_t key, uint64_t ctr) {
    return mix64(key + (ctr + 1) * kGolden);
}
// uniform in [0, n) from the low 32 bits of r
__device__ __forceinline__ uint32_t range32(uint64_t r, uint64_t n) {
    return static_cast<uint32_t>(((r & 0xFFFFFFFFull) * n) >> 32);
}

}  // namespace hc
