// Random-gather probe: the memory system's rate for the texel gathers of a
// vertex-record stream, with none of the shading arithmetic; a streaming
// probe for the device's sequential read and copy bandwidth; and an issue-rate
// probe for single vector instructions (the cost of the activation's
// exponential and reciprocal against a multiply-add, in fp32 and fp16).
//
// Both shading forms spend their time gathering one texel row per path
// vertex at the record's texel index; for uniformly random indices no
// cache line is reused, so the rate of those gathers, not the byte count,
// bounds the kernels.  This kernel reads the same records and the same rows
// and does nothing else with them: per vertex, the weight times the sum of
// the row's floats is added to a per-lane sum (so no load is dead), and
// every lane of the grid writes its sum once.  Its vertex rate is the
// ceiling the shading kernels are compared with.
//
// Layout knobs (template parameters), so that the best of several issue
// shapes can be taken as the ceiling:
//   U    vertices in flight per lane group (all records, then all rows,
//        are loaded before the first add);
//   G    lanes per row: 1 (a lane loads the whole row) or 8 (a row's
//        16-byte chunks are spread over 8 consecutive lanes);
//   CPL  16-byte chunks per lane (G * CPL >= chunks of the row).
// Rows are read in whole 16-byte chunks (row_floats rounded up to a
// multiple of 4), as the shading kernels read them.
// Vertices are taken in a grid-stride loop; records of one wave-load are
// consecutive, as in the shading kernels' pixel-major streams.

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kProbeBlock = 256;

template <int U, int G, int CPL>
__global__ __launch_bounds__(kProbeBlock) void gather_probe_kernel(const uint2* __restrict__ vtx,
                                                                   uint32_t n_vertices,
                                                                   const float* __restrict__ table,
                                                                   uint32_t n_rows, uint32_t ld,
                                                                   int chunks, float* __restrict__ out) {
    const uint64_t groups = uint64_t(gridDim.x) * (kProbeBlock / G);   // row groups in the grid
    const uint64_t g0 = uint64_t(blockIdx.x) * (kProbeBlock / G) + threadIdx.x / G;
    const int sub = threadIdx.x % G;
    float acc = 0.f;
    for (uint64_t v = g0; v < n_vertices; v += groups * U) {
        uint2 rec[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t j = v + uint64_t(u) * groups;
            rec[u] = j < n_vertices ? ldg_u2(vtx + j) : make_uint2(0u, 0u);   // weight 0 past the end
        }
        float4 row[U][CPL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float* rp = table + uint64_t(min(rec[u].x, n_rows - 1u)) * ld;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int ch = sub + c * G;
                row[u][c] = ch < chunks ? ld4(rp + 4 * ch) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < CPL; ++c) s += (row[u][c].x + row[u][c].y) + (row[u][c].z + row[u][c].w);
            acc += __uint_as_float(rec[u].y) * s;
        }
    }
    stg_f32(out + uint64_t(blockIdx.x) * kProbeBlock + threadIdx.x, acc);
}

template <int U, int G, int CPL>
hc_status launch_one(const uint2* vtx, uint32_t nv, const float* table, uint32_t n_rows, uint32_t ld,
                     int chunks, float* out, int grid, hipStream_t st) {
    hipLaunchKernelGGL((gather_probe_kernel<U, G, CPL>), dim3(grid), dim3(kProbeBlock), 0, st, vtx, nv,
                       table, n_rows, ld, chunks, out);
    return launch_status("hc_gather_probe");
}

template <int G, int CPL>
hc_status by_unroll(int unroll, const uint2* vtx, uint32_t nv, const float* table, uint32_t n_rows,
                    uint32_t ld, int chunks, float* out, int grid, hipStream_t st) {
    switch (unroll) {
        case 1: return launch_one<1, G, CPL>(vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        case 2: return launch_one<2, G, CPL>(vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        case 4: return launch_one<4, G, CPL>(vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        default: return launch_one<8, G, CPL>(vtx, nv, table, n_rows, ld, chunks, out, grid, st);
    }
}

// Streaming probe: chunk i of src (16 bytes) is read (MODE 0: its floats
// added into a per-lane sum, written once per lane) or copied to dst
// (MODE 1), in a grid-stride loop with four chunks per lane in flight.
template <int MODE>
__global__ __launch_bounds__(kProbeBlock) void stream_probe_kernel(const float* __restrict__ src,
                                                                   float* __restrict__ dst, uint64_t n16) {
    constexpr int U = 4;
    const uint64_t stride = uint64_t(gridDim.x) * kProbeBlock;
    uint64_t i = uint64_t(blockIdx.x) * kProbeBlock + threadIdx.x;
    float acc = 0.f;
    for (; i + (U - 1) * stride < n16; i += U * stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld4(src + 4 * (i + u * stride));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (MODE == 0)
                acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
            else
                st4(dst + 4 * (i + u * stride), v[u]);
        }
    }
    for (; i < n16; i += stride) {
        const float4 v = ld4(src + 4 * i);
        if (MODE == 0)
            acc += (v.x + v.y) + (v.z + v.w);
        else
            st4(dst + 4 * i, v);
    }
    if (MODE == 0) stg_f32(dst + uint64_t(blockIdx.x) * kProbeBlock + threadIdx.x, acc);
}

// Issue-rate probe: each lane runs kAluChains independent chains of
// kAluIters applications of one instruction (OP 0 fp32 multiply-add, 1
// v_exp_f32, 2 v_rcp_f32, 3 v_exp_f16, 4 v_rcp_f16, 5 packed fp16
// multiply-add), so that the SIMD issues them back to back; the chains' final
// values are summed and written once per lane (no work is dead).  The values
// themselves run to 0 / 1 / inf and do not matter: these instructions take
// the same time for any operand.
constexpr int kAluChains = HC_ALU_PROBE_CHAINS, kAluIters = HC_ALU_PROBE_ITERS;   // 16,384 instructions a lane
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

template <int OP>
__global__ __launch_bounds__(kProbeBlock) void alu_probe_kernel(float* __restrict__ out) {
    float x[kAluChains];
    _Float16 h[kAluChains];
    h2v p[kAluChains];
#pragma unroll
    for (int i = 0; i < kAluChains; ++i) {
        x[i] = float(threadIdx.x + i) * 1e-3f;
        h[i] = _Float16(x[i]);
        p[i] = h2v{h[i], _Float16(0.5f * x[i])};
    }
    const h2v pa = {_Float16(0.999f), _Float16(0.999f)}, pb = {_Float16(1e-3f), _Float16(1e-3f)};
    for (int it = 0; it < kAluIters; ++it) {
#pragma unroll
        for (int i = 0; i < kAluChains; ++i) {
            if constexpr (OP == 0) x[i] = __builtin_fmaf(x[i], 0.999f, 1e-3f);
            if constexpr (OP == 1) x[i] = __builtin_amdgcn_exp2f(x[i]);
            if constexpr (OP == 2) x[i] = __builtin_amdgcn_rcpf(x[i]);
            if constexpr (OP == 3) h[i] = __builtin_exp2f16(h[i]);
            if constexpr (OP == 4) h[i] = __builtin_amdgcn_rcph(h[i]);
            if constexpr (OP == 5) p[i] = p[i] * pa + pb;
        }
    }
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < kAluChains; ++i) sum += x[i] + float(h[i]) + float(p[i].x) + float(p[i].y);
    stg_f32(out + uint64_t(blockIdx.x) * kProbeBlock + threadIdx.x, sum);
}

}  // namespace

hc_status launch_stream_probe(const float* src, float* dst, uint64_t n16, int mode, int grid, hipStream_t st) {
    if (mode == 0)
        hipLaunchKernelGGL(stream_probe_kernel<0>, dim3(grid), dim3(kProbeBlock), 0, st, src, dst, n16);
    else
        hipLaunchKernelGGL(stream_probe_kernel<1>, dim3(grid), dim3(kProbeBlock), 0, st, src, dst, n16);
    return launch_status("hc_stream_probe");
}

hc_status launch_gather_probe(const uint2* vtx, uint32_t nv, const float* table, uint32_t n_rows,
                              uint32_t ld, int row_floats, int unroll, int lanes_per_row, float* out,
                              int grid, hipStream_t st) {
    const int chunks = (row_floats + 3) / 4;
    if (lanes_per_row == 1) {
        switch (chunks) {
            case 1: return by_unroll<1, 1>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
            case 2: return by_unroll<1, 2>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
            case 3: return by_unroll<1, 3>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
            default: return by_unroll<1, 4>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        }
    }
    switch ((chunks + 7) / 8) {
        case 1: return by_unroll<8, 1>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        case 2: return by_unroll<8, 2>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        case 3: return by_unroll<8, 3>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
        default: return by_unroll<8, 4>(unroll, vtx, nv, table, n_rows, ld, chunks, out, grid, st);
    }
}

hc_status launch_alu_probe(int op, float* out, int grid, hipStream_t st) {
    switch (op) {
        case 0: hipLaunchKernelGGL(alu_probe_kernel<0>, dim3(grid), dim3(kProbeBlock), 0, st, out); break;
        case 1: hipLaunchKernelGGL(alu_probe_kernel<1>, dim3(grid), dim3(kProbeBlock), 0, st, out); break;
        case 2: hipLaunchKernelGGL(alu_probe_kernel<2>, dim3(grid), dim3(kProbeBlock), 0, st, out); break;
        case 3: hipLaunchKernelGGL(alu_probe_kernel<3>, dim3(grid), dim3(kProbeBlock), 0, st, out); break;
        case 4: hipLaunchKernelGGL(alu_probe_kernel<4>, dim3(grid), dim3(kProbeBlock), 0, st, out); break;
        default: hipLaunchKernelGGL(alu_probe_kernel<5>, dim3(grid), dim3(kProbeBlock), 0, st, out); break;
    }
    return launch_status("hc_alu_probe");
}

}  // namespace hc
