// RGB-to-latent upsampling network (Sec. 5): z = W3 silu(W2 silu(W1 c + b1) + b2) + b3
// for every texel of an RGB asset, hidden width 128, output in the blocked RGBx
// code layout that the shading kernels read.
//
// The 128 x 128 layer is a dense contraction over texels and runs on the
// matrix cores.  Each product is computed transposed, H^T = W X^T: the
// output features are the MFMA's M dimension and 16 texels its N dimension,
// so a lane's accumulator (4 consecutive features of one texel) is exactly
// the lane's B operand for the next layer's K dimension.  Activations never
// leave registers between layers; the weights are staged once per workgroup
// in LDS in MFMA fragment order (lane l's operand at offset l), so every
// fragment read is one linear, conflict-free LDS access.
//
// Two precisions:
//   F16: fp16 operands, fp32 accumulation, v_mfma_f32_16x16x32_f16.  The K
//        order inside a 32-wide chunk is a fixed permutation of the features
//        (slots 0-3 of lane group g hold features 32c + 4g + i, slots 4-7 hold
//        32c + 16 + 4g + i); A and B use the same permutation, so the sum is
//        unchanged.
//   F32: fp32 operands, v_mfma_f32_16x16x4_f32; K chunk (16c + 4g + r) per
//        lane group g, register r.
// Layer 1 (K = 3 inputs and the bias) is one v_mfma_f32_16x16x4_f32 per 16
// features in both; the activations run on the vector ALU in fp32.

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kHidden = 128;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

typedef _Float16 hc_h8 __attribute__((ext_vector_type(8)));
typedef float hc_f4 __attribute__((ext_vector_type(4)));

struct UpArgs {
    const float* W1;  // 128 x 3
    const float* b1;
    const float* W2;  // 128 x 128
    const float* b2;
    const float* W3;  // k x 128
    const float* b3;
    int k;
    const float* rgb;
    int64_t m, ld_rgb;
    float* Z;
    int64_t ld_z;
    int64_t n_groups;  // groups of NT tiles of 16 texels
};

// With u = -log2(e) y: silu(y) = y / (1 + 2^u) = -ln(2) u / (1 + 2^u).  Both
// kernels carry s = u / (1 + 2^u) between layers: -log2(e) is folded into the
// staged layer-1 weights and bias and into the layer-2 bias, the two factors
// cancel in layer 2 (ln(2) log2(e) = 1), and layer 3 applies -ln(2) with its bias.
constexpr float kNegLog2e = -1.4426950408889634f;
constexpr float kNegLn2 = -0.6931471805599453f;

__device__ __forceinline__ float silu_log2(float u) {
    // 2^u = inf gives s = 0; 2^u = 0 gives s = u, i.e. silu(y) = y
    return u * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
}

// Feature held by slot i of lane group g in the 32-wide K chunk c (F16 order).
__device__ __forceinline__ int f16_feature(int c, int g, int i) {
    return 32 * c + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}

// Zero the padding of texel row `row` of the blocked layout (4th float of
// every slot, channels k..3B-1, columns 4B..ld_z-1), spread over lane groups.
__device__ __forceinline__ void write_padding(float* zrow, int k, int64_t ld_z, int g) {
    const int nb = (k + 2) / 3;
    for (int col = g; col < ld_z; col += 4) {
        const int b = col >> 2, j = col & 3;
        if (j == 3 || b >= nb || 3 * b + j >= k) stg_f32(zrow + col, 0.0f);
    }
}

// ------------------------------------------------------------------ F16

template <int NT, int MC3>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT > 1 ? 3 : 1))) void upsample_f16_kernel(UpArgs a) {
    __shared__ hc_h8 sW2[8 * 4 * kWave];    // [mo][c][lane]
    __shared__ hc_h8 sW3[MC3 * 4 * kWave];  // [m3][c][lane]
    __shared__ float sW1[8 * kWave];         // [mo][lane]: A operand of (w_r, w_g, w_b, b1)
    __shared__ __align__(16) float sB2[kHidden];
    __shared__ float sB3[16 * MC3];

    const int tid = threadIdx.x;
    for (int e = tid; e < 8 * 4 * kWave; e += kThreads) {
        const int lane = e % kWave, c = (e / kWave) % 4, mo = e / (4 * kWave);
        const int m = lane % 16, g = lane / 16;
        hc_h8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (_Float16)ldg_f32(a.W2 + (16 * mo + m) * kHidden + f16_feature(c, g, i));
        sW2[e] = v;
    }
    for (int e = tid; e < MC3 * 4 * kWave; e += kThreads) {
        const int lane = e % kWave, c = (e / kWave) % 4, m3 = e / (4 * kWave);
        const int row = 16 * m3 + lane % 16, g = lane / 16;
        hc_h8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            v[i] = row < a.k ? (_Float16)ldg_f32(a.W3 + row * kHidden + f16_feature(c, g, i)) : (_Float16)0.0f;
        sW3[e] = v;
    }
    for (int e = tid; e < 8 * kWave; e += kThreads) {
        // feature 16 mo + lane % 16, input component lane / 16 (3: the bias)
        const int lane = e % kWave, j = 16 * (e / kWave) + lane % 16, c = lane / 16;
        sW1[e] = kNegLog2e * (c < 3 ? ldg_f32(a.W1 + 3 * j + c) : ldg_f32(a.b1 + j));
    }
    for (int j = tid; j < kHidden; j += kThreads) sB2[j] = kNegLog2e * ldg_f32(a.b2 + j);
    for (int j = tid; j < 16 * MC3; j += kThreads) sB3[j] = j < a.k ? ldg_f32(a.b3 + j) : 0.0f;
    __syncthreads();

    const int lane = tid & (kWave - 1);
    const int g = lane / 16, n = lane % 16;
    for (int64_t grp = int64_t(blockIdx.x) * kWaves + tid / kWave; grp < a.n_groups;
         grp += int64_t(gridDim.x) * kWaves) {
        // keeps the weight reads from LDS inside the loop: hoisted out of it,
        // every fragment would stay live in registers for the whole kernel
        __asm__ volatile("" ::: "memory");
        // layer 1 on the matrix cores, K = 4: lane (g, n) brings component g of
        // texel n (g = 3: the constant 1 that takes the bias); the 16 x 16 results
        // land in the layout of layer 2's outputs, two chunks per K chunk of layer 2
        hc_h8 h1[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t texel = (grp * NT + t) * 16 + n;
            float x = g == 3 ? 1.0f : 0.0f;
            if (g < 3 && texel < a.m) x = ldg_f32(a.rgb + texel * a.ld_rgb + g);
#pragma unroll
            for (int mo = 0; mo < 8; ++mo) {
                const hc_f4 u = __builtin_amdgcn_mfma_f32_16x16x4f32(sW1[mo * kWave + lane], x,
                                                                     hc_f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) h1[t][mo >> 1][(mo & 1) * 4 + r] = (_Float16)silu_log2(u[r]);
            }
        }
        // layer 2: 8 output chunks of 16 features x 4 K chunks of 32; the chain
        // starts from the (scaled) bias, so u = W2 s1 + b2' comes out of it
        hc_h8 h2[NT][4];
#pragma unroll
        for (int mo = 0; mo < 8; ++mo) {
            const float4 b = *reinterpret_cast<const float4*>(sB2 + 16 * mo + 4 * g);
            const hc_f4 bias = {b.x, b.y, b.z, b.w};
            hc_f4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = bias;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const hc_h8 w = sW2[(mo * 4 + c) * kWave + lane];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w, h1[t][c], acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                // features 16 mo + 4 g + r of texel n: half of K chunk mo / 2
                const int half = (mo & 1) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) h2[t][mo >> 1][half + r] = (_Float16)silu_log2(acc[t][r]);
            }
        }
        // layer 3 and output
#pragma unroll
        for (int m3 = 0; m3 < MC3; ++m3) {
            hc_f4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = hc_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const hc_h8 w = sW3[(m3 * 4 + c) * kWave + lane];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w, h2[t][c], acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int64_t texel = (grp * NT + t) * 16 + n;
                if (texel >= a.m) continue;
                float* zrow = a.Z + texel * a.ld_z;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ch = 16 * m3 + 4 * g + r;
                    if (ch < a.k) stg_f32(zrow + 4 * (ch / 3) + ch % 3, fmaf(kNegLn2, acc[t][r], sB3[ch]));
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t texel = (grp * NT + t) * 16 + n;
            if (texel < a.m) write_padding(a.Z + texel * a.ld_z, a.k, a.ld_z, g);
        }
    }
}

// ------------------------------------------------------------------ F32

template <int NT, int MC3>
__global__ __launch_bounds__(kThreads) void upsample_f32_kernel(UpArgs a) {
    __shared__ float sW2[8 * 32 * kWave];  // [mo][kc * 4 + r][lane], 64 KiB
    __shared__ float sW1[8 * kWave];        // [mo][lane]: A operand of (w_r, w_g, w_b, b1)
    __shared__ __align__(16) float sB2[kHidden];

    const int tid = threadIdx.x;
    for (int e = tid; e < 8 * 32 * kWave; e += kThreads) {
        const int lane = e % kWave, ch = (e / kWave) % 32, mo = e / (32 * kWave);
        const int kc = ch / 4, r = ch % 4, m = lane % 16, g = lane / 16;
        sW2[e] = ldg_f32(a.W2 + (16 * mo + m) * kHidden + 16 * kc + 4 * g + r);
    }
    for (int e = tid; e < 8 * kWave; e += kThreads) {
        // as in the F16 kernel: scaled by -log2(e), component lane / 16 (3: the bias)
        const int lane = e % kWave, j = 16 * (e / kWave) + lane % 16, c = lane / 16;
        sW1[e] = kNegLog2e * (c < 3 ? ldg_f32(a.W1 + 3 * j + c) : ldg_f32(a.b1 + j));
    }
    for (int j = tid; j < kHidden; j += kThreads) sB2[j] = kNegLog2e * ldg_f32(a.b2 + j);
    __syncthreads();

    const int lane = tid & (kWave - 1);
    const int g = lane / 16, n = lane % 16;
    for (int64_t grp = int64_t(blockIdx.x) * kWaves + tid / kWave; grp < a.n_groups;
         grp += int64_t(gridDim.x) * kWaves) {
        // keeps the weight reads from LDS inside the loop: hoisted out of it,
        // every fragment would stay live in registers for the whole kernel
        __asm__ volatile("" ::: "memory");
        // layer 1 on the matrix cores (K = r, g, b, 1), activations s of silu_log2
        float h1[NT][8][4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t texel = (grp * NT + t) * 16 + n;
            float x = g == 3 ? 1.0f : 0.0f;
            if (g < 3 && texel < a.m) x = ldg_f32(a.rgb + texel * a.ld_rgb + g);
#pragma unroll
            for (int kc = 0; kc < 8; ++kc) {
                const hc_f4 u = __builtin_amdgcn_mfma_f32_16x16x4f32(sW1[kc * kWave + lane], x,
                                                                     hc_f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) h1[t][kc][r] = silu_log2(u[r]);
            }
        }
        float h2[NT][8][4];
#pragma unroll
        for (int mo = 0; mo < 8; ++mo) {
            const float4 b = *reinterpret_cast<const float4*>(sB2 + 16 * mo + 4 * g);
            const hc_f4 bias = {b.x, b.y, b.z, b.w};
            hc_f4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = bias;
#pragma unroll
            for (int ch = 0; ch < 32; ++ch) {
                const float w = sW2[(mo * 32 + ch) * kWave + lane];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, h1[t][ch / 4][ch % 4], acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int r = 0; r < 4; ++r) h2[t][mo][r] = silu_log2(acc[t][r]);
            }
        }
#pragma unroll
        for (int m3 = 0; m3 < MC3; ++m3) {
            const int row = 16 * m3 + n;  // A operand row of this lane
            hc_f4 acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = hc_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < 32; ++ch) {
                const int kc = ch / 4, r = ch % 4;
                const float w = row < a.k ? ldg_f32(a.W3 + row * kHidden + 16 * kc + 4 * g + r) : 0.0f;
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, h2[t][kc][r], acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int64_t texel = (grp * NT + t) * 16 + n;
                if (texel >= a.m) continue;
                float* zrow = a.Z + texel * a.ld_z;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ch = 16 * m3 + 4 * g + r;
                    if (ch < a.k) stg_f32(zrow + 4 * (ch / 3) + ch % 3, fmaf(kNegLn2, acc[t][r], ldg_f32(a.b3 + ch)));
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t texel = (grp * NT + t) * 16 + n;
            if (texel < a.m) write_padding(a.Z + texel * a.ld_z, a.k, a.ld_z, g);
        }
    }
}

// 16-texel tiles per wave per step: two tiles share each weight fragment
// read from LDS and give the matrix cores two independent accumulation chains
// (F16 with k <= 16: 112 registers, wider outputs keep one tile; F32: 196-236
// registers, 6.97 -> 6.52 ms on 4096^2 texels).
constexpr int kNT16 = 2;
constexpr int kNT32 = 2;
constexpr int kMaxGrid = 2048;

int64_t grid_for(const UpArgs& a) {
    return std::min<int64_t>(ceil_div(a.n_groups, kWaves), kMaxGrid);
}

}  // namespace

hc_status launch_upsample(const hc_mlp& net, int precision, const float* rgb, int64_t m,
                          int64_t ld_rgb, float* Z, int64_t ld_z, hipStream_t st) {
    if (m == 0) return HC_OK;
    UpArgs a;
    a.W1 = net.W1;
    a.b1 = net.b1;
    a.W2 = net.W2;
    a.b2 = net.b2;
    a.W3 = net.W3;
    a.b3 = net.b3;
    a.k = net.k;
    a.rgb = rgb;
    a.m = m;
    a.ld_rgb = ld_rgb;
    a.Z = Z;
    a.ld_z = ld_z;
    const int mc3 = int(ceil_div(net.k, 16));
    const int64_t tiles = ceil_div(m, 16);
    if (precision == HC_MLP_F16) {
        const int nt = mc3 == 1 ? kNT16 : 1;
        a.n_groups = ceil_div(tiles, nt);
        const dim3 grid(uint32_t(grid_for(a)));
        switch (mc3) {
            case 1: hipLaunchKernelGGL((upsample_f16_kernel<kNT16, 1>), grid, dim3(kThreads), 0, st, a); break;
            case 2: hipLaunchKernelGGL((upsample_f16_kernel<1, 2>), grid, dim3(kThreads), 0, st, a); break;
            default: hipLaunchKernelGGL((upsample_f16_kernel<1, 3>), grid, dim3(kThreads), 0, st, a); break;
        }
    } else {
        a.n_groups = ceil_div(tiles, kNT32);
        const dim3 grid(uint32_t(grid_for(a)));
        switch (mc3) {
            case 1: hipLaunchKernelGGL((upsample_f32_kernel<kNT32, 1>), grid, dim3(kThreads), 0, st, a); break;
            case 2: hipLaunchKernelGGL((upsample_f32_kernel<kNT32, 2>), grid, dim3(kThreads), 0, st, a); break;
            default: hipLaunchKernelGGL((upsample_f32_kernel<kNT32, 3>), grid, dim3(kThreads), 0, st, a); break;
        }
    }
    return launch_status("hc_upsample");
}

}  // namespace hc
