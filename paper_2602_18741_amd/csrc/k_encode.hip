// Linear encode z = E s (per texel / material / light) and per-pixel decode
// xyz = (T D) z, optionally s_hat = D z.  Both are tiny contractions (k x n
// with k <= 48, n <= 128) done in registers against matrices staged in LDS;
// the kernels stream rows, so HBM bandwidth bounds them.

#include "decode_common.hpp"

namespace hc {
namespace {

constexpr int kThreads = 256;

struct EncodeArgs {
    const float* E;  // k x n
    int k, n, nq;    // nq = ceil(n / 4)
    const float* S;
    int64_t m, ld_s;
    float* Z;
    int64_t ld_z;
    int rows;        // rows per block (64 or 32)
};

// Stage E into LDS as 3NB rows of nq float4 chunks, zero past k rows and
// past n samples, so a product reads a chunk of four samples at once.
template <int NB>
__device__ __forceinline__ void stage_encoder(const float* E, int k, int n, int nq, float4* s_E) {
    for (int i = threadIdx.x; i < 3 * NB * nq; i += kThreads) {
        const int c = i / nq, j = i % nq;
        float w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = (c < k && 4 * j + e < n) ? E[c * n + 4 * j + e] : 0.f;
        s_E[i] = make_float4(w[0], w[1], w[2], w[3]);
    }
}

// Encode rows [r0, r0 + nrows) (nrows <= rows per block): stage the spectra
// with coalesced float4 loads, then one thread per row accumulates the codes
// over the n samples in order.  Starts and ends with a block barrier.
template <int NB>
__device__ __forceinline__ void encode_rows(const float4* s_E, float4* s_rows, int n, int nq,
                                            const float* S, int64_t ld_s, float* Z, int64_t ld_z,
                                            int64_t r0, int nrows) {
    const int stride = nq + 1;  // float4 chunks; odd: a thread's row reads spread over banks
    const int tid = threadIdx.x;
    __syncthreads();
    for (int i = tid; i < nrows * nq; i += kThreads) {
        const int r = i / nq, c = i % nq;
        float4 v = ld4(S + (r0 + r) * ld_s + 4 * c);
        // samples past n (row padding) are not used: E is zero there, but
        // non-finite padding times zero would not be
        if (4 * c + 3 >= n) {
            if (4 * c + 1 >= n) v.y = 0.f;
            if (4 * c + 2 >= n) v.z = 0.f;
            v.w = 0.f;
        }
        s_rows[r * stride + c] = v;
    }
    __syncthreads();
    if (tid < nrows) {
        const float4* s = s_rows + tid * stride;
        // channels past k read zero rows of E (staged that way), so they stay 0
        float z[3 * NB];
#pragma unroll
        for (int c = 0; c < 3 * NB; ++c) z[c] = 0.f;
        for (int j = 0; j < nq; ++j) {
            const float4 sj = s[j];
#pragma unroll
            for (int c = 0; c < 3 * NB; ++c) {
                const float4 e = s_E[c * nq + j];
                z[c] += e.x * sj.x;
                z[c] += e.y * sj.y;
                z[c] += e.z * sj.z;
                z[c] += e.w * sj.w;
            }
        }
        float* out = Z + (r0 + tid) * ld_z;
#pragma unroll
        for (int b = 0; b < NB; ++b) st4(out + 4 * b, make_float4(z[3 * b], z[3 * b + 1], z[3 * b + 2], 0.f));
        for (int64_t f = 4 * NB; f < ld_z; f += 4) st4(out + f, make_float4(0.f, 0.f, 0.f, 0.f));
    }
}

// Long rows (n > 32).  A group of rows [r0, r0 + nrows) (nrows <= rows
// per block) is read as nrows * nq float4 chunks, chunk i by thread
// i % kThreads (coalesced), at most kLoadLong per thread, into registers;
// samples past n (row padding) are zeroed as above.
constexpr int kLoadLong = 6;  // 64 rows x 24 chunks or 32 rows x 32 chunks over 256 threads

template <int L>
__device__ __forceinline__ void load_group(const float* S, int64_t ld_s, int n, int nq, int64_t r0, int nrows,
                                           float4 (&v)[L]) {
    const int total = nrows * nq;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int i = int(threadIdx.x) + t * kThreads;
        if (i < total) {
            const int r = i / nq, c = i % nq;
            float4 x = ld4(S + (r0 + r) * ld_s + 4 * c);
            if (4 * c + 3 >= n) {
                if (4 * c + 1 >= n) x.y = 0.f;
                if (4 * c + 2 >= n) x.z = 0.f;
                x.w = 0.f;
            }
            v[t] = x;
        }
    }
}

template <int L>
__device__ __forceinline__ void put_group(float4* s_rows, int nq, int nrows, const float4 (&v)[L]) {
    const int stride = nq + 1;  // float4 chunks; odd: a row's reads spread over banks
    const int total = nrows * nq;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int i = int(threadIdx.x) + t * kThreads;
        if (i < total) s_rows[(i / nq) * stride + i % nq] = v[t];
    }
}

// Codes of the staged group of long rows: kThreads / rows threads share a
// row, each accumulating its channels (q, q + that count, ...) over the
// samples in order (each channel's sums as in encode_rows, so the results
// are the same bits); the codes go through LDS (s_z, rows x NB float4) to
// whole-row float4 stores.  Called with the group staged and a barrier
// passed; ends with the stores.
template <int NB>
__device__ __forceinline__ void encode_group(const float4* s_E, const float4* s_rows, float4* s_z, int nq,
                                             int rows, float* Z, int64_t ld_z, int64_t r0, int nrows) {
    const int tid = threadIdx.x;
    // at least 4 threads per row (rows <= 64): at most ceil(3NB / 4) channels each
    constexpr int kChan = (3 * NB + 3) / 4;
    const int tpr = kThreads / rows;
    const int r = tid / tpr, q = tid % tpr;
    if (r < nrows) {
        const float4* s = s_rows + r * (nq + 1);
        // channels past k read zero rows of E (staged that way), so they stay 0
        float z[kChan];
#pragma unroll
        for (int i = 0; i < kChan; ++i) z[i] = 0.f;
        for (int j = 0; j < nq; ++j) {
            const float4 sj = s[j];
#pragma unroll
            for (int i = 0; i < kChan; ++i) {
                const int c = q + i * tpr;
                if (c < 3 * NB) {
                    const float4 e = s_E[c * nq + j];
                    z[i] += e.x * sj.x;
                    z[i] += e.y * sj.y;
                    z[i] += e.z * sj.z;
                    z[i] += e.w * sj.w;
                }
            }
        }
        float* zr = reinterpret_cast<float*>(s_z + r * NB);
#pragma unroll
        for (int i = 0; i < kChan; ++i) {
            const int c = q + i * tpr;
            if (c < 3 * NB) zr[4 * (c / 3) + c % 3] = z[i];
        }
        for (int b = q; b < NB; b += tpr) zr[4 * b + 3] = 0.f;
    }
    __syncthreads();
    // the row's float4 chunks by its threads in turn (consecutive lanes,
    // consecutive chunks): the codes, then zero columns up to the stride
    if (r < nrows) {
        float* out = Z + (r0 + r) * ld_z;
        for (int64_t f = q; 4 * f < ld_z; f += tpr)
            st4(out + 4 * f, f < NB ? s_z[r * NB + f] : make_float4(0.f, 0.f, 0.f, 0.f));
    }
}

template <int NB>
__global__ __launch_bounds__(kThreads) void encode_kernel(EncodeArgs a) {
    extern __shared__ float4 smem[];
    float4* s_E = smem + a.rows * (a.nq + 1);
    stage_encoder<NB>(a.E, a.k, a.n, a.nq, s_E);
    const int64_t r0 = int64_t(blockIdx.x) * a.rows;
    const int nrows = int(min<int64_t>(a.rows, a.m - r0));
    encode_rows<NB>(s_E, smem, a.n, a.nq, a.S, a.ld_s, a.Z, a.ld_z, r0, nrows);
}

// Long rows: a persistent grid (the workgroups the device holds at once),
// each staging E once and walking the row groups blockIdx.x, + gridDim.x,
// ...; the next group's rows are loaded into registers while the current
// one is encoded.
template <int NB>
__global__ __launch_bounds__(kThreads) void encode_long_kernel(EncodeArgs a) {
    extern __shared__ float4 smem[];
    float4* s_E = smem + a.rows * (a.nq + 1);
    float4* s_z = s_E + 3 * NB * a.nq;
    stage_encoder<NB>(a.E, a.k, a.n, a.nq, s_E);
    const int64_t groups = (a.m + a.rows - 1) / a.rows;
    int64_t g = blockIdx.x;
    float4 v[kLoadLong];
    if (g < groups) load_group(a.S, a.ld_s, a.n, a.nq, g * a.rows, int(min<int64_t>(a.rows, a.m - g * a.rows)), v);
    for (; g < groups; g += gridDim.x) {
        const int64_t r0 = g * a.rows;
        const int nrows = int(min<int64_t>(a.rows, a.m - r0));
        __syncthreads();  // E staged; the previous group's reads of LDS are done
        put_group(smem, a.nq, nrows, v);
        __syncthreads();
        const int64_t gn = g + gridDim.x;
        if (gn < groups)
            load_group(a.S, a.ld_s, a.n, a.nq, gn * a.rows, int(min<int64_t>(a.rows, a.m - gn * a.rows)), v);
        encode_group<NB>(s_E, smem, s_z, a.nq, a.rows, a.Z, a.ld_z, r0, nrows);
    }
}

// Persistent launch over an encode job table (rows [begin, end) of one
// spectra array each); block b takes jobs b, b + grid, ...
template <int NB, bool LONG>
__global__ __launch_bounds__(kThreads) void encode_jobs_kernel(const hc_encode_job* __restrict__ jobs,
                                                               const int32_t* __restrict__ n_jobs_dev,
                                                               int max_jobs,
                                                               const float* E, int k, int n, int rows) {
    extern __shared__ float4 smem[];
    const int nq = (n + 3) / 4;
    float4* s_E = smem + rows * (nq + 1);
    float4* s_z = s_E + 3 * NB * nq;
    stage_encoder<NB>(E, k, n, nq, s_E);
    const int n_jobs = min(*n_jobs_dev, max_jobs);
    for (int j = blockIdx.x; j < n_jobs; j += gridDim.x) {
        const hc_encode_job job = jobs[j];
        for (int64_t r0 = job.begin; r0 < job.end; r0 += rows) {
            const int nrows = int(min<int64_t>(rows, job.end - r0));
            if constexpr (LONG) {
                float4 v[kLoadLong];
                load_group(job.S, job.ld_s, n, nq, r0, nrows, v);
                __syncthreads();  // E staged; the previous rows' reads of LDS are done
                put_group(smem, nq, nrows, v);
                __syncthreads();
                encode_group<NB>(s_E, smem, s_z, nq, rows, job.Z, job.ld_z, r0, nrows);
            } else {
                encode_rows<NB>(s_E, smem, n, nq, job.S, job.ld_s, job.Z, job.ld_z, r0, nrows);
            }
        }
    }
}

struct DecodeArgs {
    const float* D;  // n x k
    const float* T;  // 3 x n
    int n, k, nb;
    const float* zimg;
    int64_t n_pixels, ld_z;
    float* xyz;
    float* spectra;
    int64_t ld_s;
};

// M = T D (3 x 3NB, zero columns past k) into LDS; D too when spectra are
// requested.
template <int NB>
__device__ __forceinline__ void stage_decoder(const float* D, const float* T, int n, int k, float* s_M,
                                              float* s_D) {
    for (int e = threadIdx.x; e < 9 * NB; e += kThreads) s_M[e] = decoder_entry<NB>(D, T, n, k, e);
    if (s_D)
        for (int e = threadIdx.x; e < n * k; e += kThreads) s_D[e] = D[e];
}

template <int NB>
__device__ __forceinline__ void decode_pixel(const float* s_M, const float* s_D, int n, int k,
                                             const float* zimg, int64_t ld_z, float* xyz, float* spectra,
                                             int64_t ld_s, int64_t q) {
    float z[3 * NB];
    const float* row = zimg + q * ld_z;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float4 v = ld4(row + 4 * b);
        z[3 * b] = v.x;
        z[3 * b + 1] = v.y;
        z[3 * b + 2] = v.z;
    }
    float x, y, w;
    decode_dot<NB>(s_M, z, x, y, w);
    float* o = xyz + q * 3;
    stg_f32(o + 0, x);
    stg_f32(o + 1, y);
    stg_f32(o + 2, w);
    if (spectra) {
        float* sp = spectra + q * ld_s;
        for (int i = 0; i < n; ++i) {
            float acc = 0.f;
            for (int c = 0; c < k; ++c) acc += s_D[i * k + c] * z[c];
            stg_f32(sp + i, acc);
        }
    }
}

// decode_pixels<NB>() pixels per thread (consecutive blocks of kThreads
// pixels), so a workgroup's set-up of M is shared by that many pixels; fewer
// for wide codes, whose preloaded rows would not fit the registers.
template <int NB>
constexpr int decode_pixels() { return NB <= 4 ? 8 : (NB <= 8 ? 4 : 2); }

template <int NB>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs a) {
    constexpr int kDecodePixels = decode_pixels<NB>();
    __shared__ float s_M[3 * kMaxK];
    extern __shared__ float s_D[];  // n x k, only when spectra are requested
    const int64_t q0 = int64_t(blockIdx.x) * kThreads * kDecodePixels + threadIdx.x;
    if (!a.spectra) {
        // the latent pixels of all kDecodePixels pixels are in flight while
        // M is staged (pixels past the image read pixel 0 and are dropped)
        float4 zv[kDecodePixels][NB];
#pragma unroll
        for (int i = 0; i < kDecodePixels; ++i) {
            const int64_t q = q0 + int64_t(i) * kThreads;
            const float* row = a.zimg + (q < a.n_pixels ? q : 0) * a.ld_z;
#pragma unroll
            for (int b = 0; b < NB; ++b) zv[i][b] = ld4(row + 4 * b);
        }
        stage_decoder<NB>(a.D, a.T, a.n, a.k, s_M, nullptr);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kDecodePixels; ++i) {
            const int64_t q = q0 + int64_t(i) * kThreads;
            if (q >= a.n_pixels) break;
            float z[3 * NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                z[3 * b] = zv[i][b].x;
                z[3 * b + 1] = zv[i][b].y;
                z[3 * b + 2] = zv[i][b].z;
            }
            float x, y, w;
            decode_dot<NB>(s_M, z, x, y, w);
            float* o = a.xyz + q * 3;
            stg_f32(o + 0, x);
            stg_f32(o + 1, y);
            stg_f32(o + 2, w);
        }
        return;
    }
    stage_decoder<NB>(a.D, a.T, a.n, a.k, s_M, s_D);
    __syncthreads();
    for (int i = 0; i < kDecodePixels; ++i) {
        const int64_t q = q0 + int64_t(i) * kThreads;
        if (q >= a.n_pixels) return;
        decode_pixel<NB>(s_M, s_D, a.n, a.k, a.zimg, a.ld_z, a.xyz, a.spectra, a.ld_s, q);
    }
}

// Persistent launch over a tile table: each tile's pixels of frames[f].image
// are decoded to frames[f].xyz.
template <int NB>
__global__ __launch_bounds__(kThreads) void decode_tiles_kernel(const hc_frame* __restrict__ frames,
                                                                int n_frames,
                                                                const hc_tile* __restrict__ tiles,
                                                                const int32_t* __restrict__ n_tiles_dev,
                                                                int max_tiles,
                                                                const float* D, int n, int k,
                                                                const float* T) {
    __shared__ float s_M[3 * kMaxK];
    stage_decoder<NB>(D, T, n, k, s_M, nullptr);
    __syncthreads();
    const int n_tiles = min(*n_tiles_dev, max_tiles);
    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const hc_tile tile = tiles[t];
        if (tile.frame < 0 || tile.frame >= n_frames) continue;
        const hc_frame& fr = frames[tile.frame];
        const int64_t begin = tile.begin < 0 ? 0 : tile.begin;
        const int64_t end = tile.end > fr.n_pixels ? fr.n_pixels : tile.end;
        for (int64_t q = begin + threadIdx.x; q < end; q += kThreads)
            decode_pixel<NB>(s_M, nullptr, n, k, fr.image, fr.ld_image, fr.xyz, nullptr, 0, q);
    }
}

// M = T D written out (3 x 3NB, zero columns past k), for the shading
// kernel's fused decode.  One workgroup: D and T are staged in LDS with one
// load per thread in flight, so each entry's chain of n multiply-adds reads
// LDS instead of waiting on global loads (the same operands, so the same
// bits as the decode kernels' staging).
template <int NB>
__global__ __launch_bounds__(kThreads) void decode_matrix_kernel(const float* D, const float* T, int n, int k,
                                                                 float* M) {
    __shared__ float s_D[kMaxN * kMaxK];
    __shared__ float s_T[3 * kMaxN];
    for (int i = threadIdx.x; i < n * k; i += kThreads) s_D[i] = D[i];
    for (int i = threadIdx.x; i < 3 * n; i += kThreads) s_T[i] = T[i];
    __syncthreads();
    for (int e = threadIdx.x; e < 9 * NB; e += kThreads) stg_f32(M + e, decoder_entry<NB>(s_D, s_T, n, k, e));
}

#define HC_NB_CASES(M) \
    M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)

// Rows longer than 32 samples take the pipelined kernels.  Rows per block:
// 64 (short rows: one thread per row; long ones: four) up to 96 samples, 32
// (eight threads per row) beyond.
bool long_rows(int nq) { return nq > 8; }
int rows_per_block(int nq) { return nq <= 24 ? 64 : 32; }

size_t encode_lds(int rows, int nq, int nb, bool lng) {
    return (size_t(rows) * (nq + 1) + size_t(3 * nb) * nq + (lng ? size_t(rows) * nb : 0)) * sizeof(float4);
}

}  // namespace

hc_status launch_encode(const float* E, int k, int n, const float* S, int64_t m, int64_t ld_s,
                        float* Z, int64_t ld_z, hipStream_t st) {
    EncodeArgs a;
    a.E = E;
    a.k = k;
    a.n = n;
    a.nq = (n + 3) / 4;
    a.S = S;
    a.m = m;
    a.ld_s = ld_s;
    a.Z = Z;
    a.ld_z = ld_z;
    a.rows = rows_per_block(a.nq);
    const int nb = (k + 2) / 3;
    const bool lng = long_rows(a.nq);
    const size_t lds = encode_lds(a.rows, a.nq, nb, lng);
    const int64_t groups = ceil_div(m, a.rows);
    if (!lng && groups > 0x7FFFFFFF) {
        set_error("hc_encode: too many rows for one launch");
        return HC_ESHAPE;
    }
    switch (nb) {
#define HC_ENC(NB)                                                                                  \
    case NB:                                                                                        \
        if (!lng) {                                                                                 \
            hipLaunchKernelGGL(encode_kernel<NB>, dim3(uint32_t(groups)), dim3(kThreads), lds, st, a); \
        } else {                                                                                    \
            const int res = resident_grid(encode_long_kernel<NB>, kThreads, lds, "hc_encode");     \
            if (res <= 0) return HC_EDEVICE;                                                        \
            const int grid = int(std::max<int64_t>(1, std::min<int64_t>(groups, res)));             \
            hipLaunchKernelGGL(encode_long_kernel<NB>, dim3(grid), dim3(kThreads), lds, st, a);     \
        }                                                                                           \
        break;
        HC_NB_CASES(HC_ENC)
#undef HC_ENC
        default:
            set_error("hc_encode: k=%d unsupported", k);
            return HC_EUNSUPPORTED;
    }
    return launch_status("hc_encode");
}

hc_status launch_decode(const float* D, int n, int k, const float* T, const float* zimg,
                        int64_t n_pixels, int64_t ld_zimg, float* xyz, float* spectra,
                        int64_t ld_spectra, hipStream_t st) {
    DecodeArgs a;
    a.D = D;
    a.T = T;
    a.n = n;
    a.k = k;
    a.nb = (k + 2) / 3;
    a.zimg = zimg;
    a.n_pixels = n_pixels;
    a.ld_z = ld_zimg;
    a.xyz = xyz;
    a.spectra = spectra;
    a.ld_s = ld_spectra;
    const size_t lds = spectra ? size_t(n) * k * sizeof(float) : 0;
    // the fewest pixels per thread (2) bounds the grid
    if (ceil_div(n_pixels, int64_t(kThreads) * 2) > 0x7FFFFFFF) {
        set_error("hc_decode_xyz: too many pixels for one launch");
        return HC_ESHAPE;
    }
    switch (a.nb) {
#define HC_DEC(NB)                                                                               \
    case NB: {                                                                                   \
        const int64_t blocks = ceil_div(n_pixels, int64_t(kThreads) * decode_pixels<NB>());      \
        hipLaunchKernelGGL(decode_kernel<NB>, dim3(uint32_t(blocks)), dim3(kThreads), lds, st, a); \
        break;                                                                                   \
    }
        HC_NB_CASES(HC_DEC)
#undef HC_DEC
        default:
            set_error("hc_decode_xyz: k=%d unsupported", k);
            return HC_EUNSUPPORTED;
    }
    return launch_status("hc_decode_xyz");
}

hc_status launch_decode_matrix(const float* D, int n, int k, const float* T, float* M, hipStream_t st) {
    switch ((k + 2) / 3) {
#define HC_DECM(NB) \
    case NB: hipLaunchKernelGGL(decode_matrix_kernel<NB>, dim3(1), dim3(kThreads), 0, st, D, T, n, k, M); break;
        HC_NB_CASES(HC_DECM)
#undef HC_DECM
        default:
            set_error("hc_decode_matrix: k=%d unsupported", k);
            return HC_EUNSUPPORTED;
    }
    return launch_status("hc_decode_matrix");
}

hc_status launch_encode_jobs(const hc_encode_job* jobs, const int32_t* n_jobs, int max_jobs,
                             const float* E, int k, int n, int grid, hipStream_t st) {
    const int nq = (n + 3) / 4;
    const int rows = rows_per_block(nq);
    const int nb = (k + 2) / 3;
    const size_t lds = encode_lds(rows, nq, nb, long_rows(nq));
    switch (nb) {
#define HC_ENCJ_L(NB, L)                                                                             \
    {                                                                                                \
        const int g = tile_grid(grid, encode_jobs_kernel<NB, L>, kThreads, lds, "hc_encode_jobs");   \
        if (g <= 0) return HC_EDEVICE;                                                               \
        hipLaunchKernelGGL((encode_jobs_kernel<NB, L>), dim3(g), dim3(kThreads), lds, st, jobs,      \
                           n_jobs, max_jobs, E, k, n, rows);                                         \
    }
#define HC_ENCJ(NB)                                                                                  \
    case NB:                                                                                         \
        if (long_rows(nq))                                                                           \
            HC_ENCJ_L(NB, true)                                                                      \
        else                                                                                         \
            HC_ENCJ_L(NB, false)                                                                     \
        break;
        HC_NB_CASES(HC_ENCJ)
#undef HC_ENCJ
#undef HC_ENCJ_L
        default:
            set_error("hc_encode_jobs: k=%d unsupported", k);
            return HC_EUNSUPPORTED;
    }
    return launch_status("hc_encode_jobs");
}

hc_status launch_decode_tiles(const hc_frame* frames, int n_frames, const hc_tile* tiles,
                              const int32_t* n_tiles, int max_tiles, const float* D, int n, int k,
                              const float* T, int grid, hipStream_t st) {
    switch ((k + 2) / 3) {
#define HC_DECT(NB)                                                                                  \
    case NB: {                                                                                       \
        const int g = tile_grid(grid, decode_tiles_kernel<NB>, kThreads, 0, "hc_decode_tiles");      \
        if (g <= 0) return HC_EDEVICE;                                                               \
        hipLaunchKernelGGL(decode_tiles_kernel<NB>, dim3(g), dim3(kThreads), 0, st, frames, n_frames, \
                           tiles, n_tiles, max_tiles, D, n, k, T);                                   \
        break;                                                                                       \
    }
        HC_NB_CASES(HC_DECT)
#undef HC_DECT
        default:
            set_error("hc_decode_tiles: k=%d unsupported", k);
            return HC_EUNSUPPORTED;
    }
    return launch_status("hc_decode_tiles");
}

}  // namespace hc
