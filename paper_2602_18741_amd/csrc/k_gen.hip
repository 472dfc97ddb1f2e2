// Synthetic light-path records and random indices from a counter-based
// generator: SplitMix64's output function (Steele, Lea and Flood, OOPSLA
// 2014) applied to key + (counter + 1) * 0x9E3779B97F4A7C15, with
// key = mix64(mix64(seed) + stream).  Any path is reproducible on its own.

#include "counter_rng.hpp"
#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 4;                      // items per thread in the scan
constexpr int kScanTile = kThreads * kScanItems;   // pixels per scan block

struct GenArgs {
    int64_t n_pixels;
    int spp, l_min, l_span;  // l_span = l_max - l_min + 1
    uint32_t n_illum;
    uint64_t n_tex;
    uint64_t key_path, key_vtx;
};

__device__ __forceinline__ uint32_t path_length(const GenArgs& g, uint64_t p) {
    return uint32_t(g.l_min) + range32(rand64(g.key_path, p), uint64_t(g.l_span));
}

// Lane-per-path mapping shared by the two record kernels: a pixel's paths are
// `seg` consecutive lanes (spp rounded up to a power of two, at most 64; more
// samples loop over rounds of seg paths), `pw` pixels per wavefront.
struct Seg {
    int seg, pw, rounds;
};

Seg seg_of(int spp) {
    Seg s;
    s.seg = 1;
    while (s.seg < spp && s.seg < kWave) s.seg <<= 1;
    s.pw = kWave / s.seg;
    s.rounds = int(ceil_div(spp, s.seg));
    return s;
}

// Both record kernels run a fixed grid: wavefront w takes the pixel groups
// w, w + (wavefronts in the grid), ... (a group is `pw` pixels), so the
// per-wavefront set-up is paid once per many groups.

// hdr of every path (stores coalesced across the lanes), and each pixel's
// vertex count into pix_first (sum over the pixel's lanes by xor shuffles)
__global__ __launch_bounds__(kThreads) void gen_headers_kernel(GenArgs g, Seg s, uint32_t* hdr,
                                                               uint32_t* counts) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = int64_t(gridDim.x) * (kThreads / kWave);
    const int j0 = lane % s.seg;
    for (int64_t wave = (int64_t(blockIdx.x) * kThreads + threadIdx.x) / kWave; wave * s.pw < g.n_pixels;
         wave += waves) {
        const int64_t q = wave * s.pw + lane / s.seg;
        const bool pix_ok = q < g.n_pixels;
        uint32_t sum = 0;
        for (int r = 0; r < s.rounds; ++r) {
            const int j = j0 + r * s.seg;
            if (pix_ok && j < g.spp) {
                const uint64_t p = uint64_t(q) * g.spp + j;
                const uint64_t rr = rand64(g.key_path, p);
                const uint32_t len = uint32_t(g.l_min) + range32(rr, uint64_t(g.l_span));
                const uint32_t light = static_cast<uint32_t>(((rr >> 32) * g.n_illum) >> 32);
                hdr[p] = light | (len << 24);
                sum += len;
            }
        }
        for (int m = 1; m < s.seg; m <<= 1) sum += __shfl_xor(sum, m, kWave);
        if (pix_ok && j0 == 0) counts[q] = sum;
    }
}

// Exclusive scan of the per-pixel counts (reduce, scan of block sums, scan).
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* s_tmp, uint64_t& total) {
    // inclusive scan inside the wave
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint64_t x = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_tmp[wave] = x;
    __syncthreads();
    uint64_t off = 0;
    for (int w = 0; w < wave; ++w) off += s_tmp[w];
    total = 0;
    for (int w = 0; w < kThreads / kWave; ++w) total += s_tmp[w];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* counts, int64_t n,
                                                               uint64_t* block_sums) {
    __shared__ uint64_t s_tmp[kThreads / kWave];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    uint64_t v = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) v += counts[base + i];
    uint64_t total;
    block_exclusive_scan(v, s_tmp, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// single workgroup: exclusive scan of the block sums in place, total out
__global__ __launch_bounds__(kThreads) void scan_blocks_kernel(uint64_t* block_sums, int64_t nb,
                                                               uint64_t* total_out) {
    __shared__ uint64_t s_tmp[kThreads / kWave];
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        const int64_t b = b0 + threadIdx.x;
        const uint64_t v = b < nb ? block_sums[b] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(v, s_tmp, total);
        if (b < nb) block_sums[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(uint32_t* counts, int64_t n,
                                                              const uint64_t* block_offsets) {
    __shared__ uint64_t s_tmp[kThreads / kWave];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    uint32_t c[kScanItems];
    uint64_t v = 0;
    for (int i = 0; i < kScanItems; ++i) {
        c[i] = (base + i < n) ? counts[base + i] : 0u;
        v += c[i];
    }
    uint64_t total;
    uint64_t run = block_offsets[blockIdx.x] + block_exclusive_scan(v, s_tmp, total);
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) counts[base + i] = static_cast<uint32_t>(run);
        run += c[i];
    }
}

// One vertex record of path p: texel and weight from the vertex's own draw.
__device__ __forceinline__ uint2 vertex_record(const GenArgs& g, uint64_t p, uint32_t v) {
    const uint64_t rr = rand64(g.key_vtx, p * 256u + v);
    const uint32_t texel = range32(rr, g.n_tex);
    const float w = float(uint32_t(rr >> 40)) * (1.0f / 16777216.0f);
    return make_uint2(texel, __float_as_uint(w));
}

// Lane 0's value of a 64-bit integer.  readfirstlane returns a signed int:
// each half goes through uint32_t before widening, so a low half of 2^31 or
// more is not sign-extended into the high half.
__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
    return (uint64_t(hi) << 32) | lo;
}

// Vertex records the flat path of a round may hold per wavefront (one byte
// of lane id each in LDS); rounds with more take the lane-per-path path.
constexpr int kOwnerCap = 2048;

// LDS written by other lanes of the same wavefront is read below: wait for
// the LDS operations in flight (lgkmcnt 0, other counters untouched) and keep
// the compiler from moving memory operations across.
__device__ __forceinline__ void wave_lds_sync() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

// A round's paths (one per lane) own consecutive record ranges: a path's
// first record is its pixel's first record plus the lengths of the pixel's
// earlier paths (exclusive scan over the pixel's lanes), and the pixels of a
// wavefront follow each other.  Records are made lane-per-record over that
// flat range, so the stores of a wavefront are contiguous: each lane marks
// its records with its lane id in LDS, then lane i makes records i, i + 64, ...
__global__ __launch_bounds__(kThreads) void gen_vertices_kernel(GenArgs g, Seg s, const uint32_t* pix_first,
                                                                uint32_t* vtx, uint64_t n_vertices) {
    __shared__ uint8_t s_owner[kThreads / kWave][kOwnerCap];
    __shared__ uint32_t s_off[kThreads / kWave][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t waves = int64_t(gridDim.x) * (kThreads / kWave);
    const int seg_log2 = __builtin_ctz(unsigned(s.seg));
    const int j0 = lane & (s.seg - 1);
    const int last = (lane & ~(s.seg - 1)) + s.seg - 1;  // the segment's last lane
    uint2* out = reinterpret_cast<uint2*>(vtx);
    for (int64_t wave = (int64_t(blockIdx.x) * kThreads + threadIdx.x) / kWave; wave * s.pw < g.n_pixels;
         wave += waves) {
        const int64_t q = wave * s.pw + (lane >> seg_log2);
        const bool pix_ok = q < g.n_pixels;
        uint64_t next = pix_ok ? pix_first[q] : 0;
        for (int r = 0; r < s.rounds; ++r) {
            const int j = j0 + r * s.seg;
            const bool live = pix_ok && j < g.spp;
            const uint64_t p = uint64_t(q) * g.spp + j;
            const uint32_t len = live ? path_length(g, p) : 0u;
            uint32_t incl = len;
            for (int d = 1; d < s.seg; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d, kWave);
                if (j0 >= d) incl += y;
            }
            const uint32_t total = __shfl(incl, last, kWave);
            const uint64_t first = next + (incl - len);
            next += total;
            // the round's flat range starts at lane 0's first record (lane 0 is
            // always a live path) and ends at the largest end over the lanes
            const uint64_t base = first_lane_u64(first);
            const uint32_t off = pix_ok ? uint32_t(first - base) : 0u;  // past the frame: no records
            uint32_t span = off + len;
            for (int m = 1; m < kWave; m <<= 1) span = max(span, uint32_t(__shfl_xor(int(span), m, kWave)));
            if (span <= uint32_t(kOwnerCap)) {
                s_off[wv][lane] = off;
                for (uint32_t v = 0; v < len; ++v) s_owner[wv][off + v] = uint8_t(lane);
                wave_lds_sync();
                for (uint32_t i = lane; i < span; i += kWave) {
                    const int pl = s_owner[wv][i];
                    const uint32_t v = i - s_off[wv][pl];
                    const uint64_t pq = uint64_t(wave * s.pw + (pl >> seg_log2));
                    const uint64_t pp = pq * g.spp + ((pl & (s.seg - 1)) + r * s.seg);
                    const uint64_t jv = base + i;
                    if (jv < n_vertices) out[jv] = vertex_record(g, pp, v);
                }
                wave_lds_sync();  // the next round overwrites the maps
            } else {
                for (uint32_t v = 0; v < len; ++v) {
                    const uint64_t jv = first + v;
                    if (jv >= n_vertices) break;
                    out[jv] = vertex_record(g, p, v);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void gen_indices_kernel(uint64_t key, uint64_t ctr0,
                                                               const int64_t* scale, int64_t count,
                                                               uint64_t n, uint32_t* out) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= count) return;
    const uint64_t base = ctr0 + (scale ? uint64_t(*scale) * uint64_t(count) : 0ull);
    out[i] = range32(rand64(key, base + uint64_t(i)), n);
}

// Workgroups of a record kernel: enough for `groups` pixel groups, at most
// kGenRounds times the workgroups the device holds at once.
constexpr int kGenRounds = 4;

template <typename K>
int gen_grid(int64_t groups, K kernel, size_t lds, const char* what) {
    const int res = resident_grid(kernel, kThreads, lds, what);
    if (res <= 0) return 0;
    const int64_t want = ceil_div(groups, kThreads / kWave);
    return int(std::max<int64_t>(1, std::min<int64_t>(want, int64_t(kGenRounds) * res)));
}

GenArgs make_args(const hc_path_gen& g) {
    GenArgs a;
    a.n_pixels = g.n_pixels;
    a.spp = g.spp;
    a.l_min = g.l_min;
    a.l_span = g.l_max - g.l_min + 1;
    a.n_illum = static_cast<uint32_t>(g.n_illum);
    a.n_tex = static_cast<uint64_t>(g.n_tex);
    a.key_path = stream_key(g.seed, 1);
    a.key_vtx = stream_key(g.seed, 2);
    return a;
}

}  // namespace

size_t gen_workspace_size(int64_t n_pixels) {
    return size_t(ceil_div(n_pixels, kScanTile) + 1) * sizeof(uint64_t);
}

hc_status launch_gen_headers(const hc_path_gen& g, uint32_t* hdr, uint32_t* pix_first,
                             uint64_t* n_vertices, void* ws, size_t, hipStream_t st) {
    const GenArgs a = make_args(g);
    uint64_t* block_sums = static_cast<uint64_t*>(ws);
    const int64_t nb = ceil_div(g.n_pixels, kScanTile);
    if (g.n_pixels > 0) {
        const Seg sg = seg_of(g.spp);
        const int grid = gen_grid(ceil_div(g.n_pixels, sg.pw), gen_headers_kernel, 0, "hc_gen_path_headers");
        if (grid <= 0) return HC_EDEVICE;
        hipLaunchKernelGGL(gen_headers_kernel, dim3(grid), dim3(kThreads), 0, st, a, sg, hdr, pix_first);
        hc_status s = launch_status("hc_gen_path_headers");
        if (s != HC_OK) return s;
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(uint32_t(nb)), dim3(kThreads), 0, st, pix_first,
                           g.n_pixels, block_sums);
        s = launch_status("hc_gen_path_headers");
        if (s != HC_OK) return s;
    }
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kThreads), 0, st, block_sums, nb,
                       reinterpret_cast<uint64_t*>(n_vertices));
    hc_status s = launch_status("hc_gen_path_headers");
    if (s != HC_OK || g.n_pixels == 0) return s;
    hipLaunchKernelGGL(scan_apply_kernel, dim3(uint32_t(nb)), dim3(kThreads), 0, st, pix_first,
                       g.n_pixels, block_sums);
    return launch_status("hc_gen_path_headers");
}

hc_status launch_gen_vertices(const hc_path_gen& g, const uint32_t* pix_first, uint32_t* vtx,
                              int64_t n_vertices, hipStream_t st) {
    const GenArgs a = make_args(g);
    if (g.n_pixels == 0) return HC_OK;
    const Seg sg = seg_of(g.spp);
    const int grid = gen_grid(ceil_div(g.n_pixels, sg.pw), gen_vertices_kernel, 0, "hc_gen_path_vertices");
    if (grid <= 0) return HC_EDEVICE;
    hipLaunchKernelGGL(gen_vertices_kernel, dim3(grid), dim3(kThreads), 0, st, a, sg, pix_first, vtx,
                       uint64_t(n_vertices));
    return launch_status("hc_gen_path_vertices");
}

hc_status launch_gen_indices(uint64_t seed, uint64_t ctr0, const int64_t* scale, int64_t count,
                             int64_t n, uint32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(gen_indices_kernel, dim3(uint32_t(ceil_div(count, kThreads))), dim3(kThreads), 0,
                       st, stream_key(seed, kIndexStream), ctr0, scale, count, uint64_t(n), out);
    return launch_status("hc_gen_indices");
}

}  // namespace hc
