// Training step of the upsampling network (Sec. 5.2): loss, hand-written
// backward and AdamW with global-norm gradient clipping, on a batch of
// (RGB, code) pairs gathered by index or drawn from the counter-based
// generator inside kernel 1.  Deterministic: fixed summation orders, no
// floating-point atomics.
//
//   1. partials: a workgroup (at most 256: one partial row each) takes
//                tiles of 16 samples; the layer products of the tile, forward
//                and backward, and the weight gradients summed over its
//                samples are 16x16x4 fp32 matrix-core products with W3 and
//                the tile's activations in LDS and each wavefront's W2
//                fragments in registers (details at the kernel); the
//                gradient sums stay in registers across tiles.
//   2. reduce  : a lane per parameter sums the partial rows in a fixed order
//                (float64, sixteen row loads in flight), divides by N, writes
//                the gradient, and each block writes its sum of squares;
//                block 0 also sums the per-row losses (a wavefront butterfly)
//                and increments the step counter, after kernel 1's draw.
//   3. adamw   : every block forms the global gradient norm from the block
//                sums (same order everywhere), the clipping factor
//                min(1, max_norm / (norm + 1e-6)), then per parameter the
//                decoupled weight decay and the Adam update.

#include <cmath>

#include "counter_rng.hpp"
#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kH = 128;            // hidden width
constexpr int kThreads = 256;      // reduce and AdamW kernels
constexpr int kTS = 16;            // samples of a tile (the N of every 16 x 16 x 4 product)
constexpr int kPThreads = 512;     // partials kernel: 8 wavefronts, wave w owns hidden rows 16w..16w+15
constexpr int kPWaves = kPThreads / 64;
static_assert(kPWaves * 16 == kH, "one 16-row block of the hidden layer per wavefront");
// LDS row strides (floats): W2 and W3 rows 4 banks apart, so the 16 rows x 4
// columns of a forward operand read are conflict-free; activations are
// [feature][sample] with 17 floats per feature row
constexpr int kRS = kH + 4;
constexpr int kAS = kTS + 1;
constexpr int kMaxRows = 256;      // partial rows (workgroups of kernel 1)
static_assert(kMaxRows <= kThreads, "one workgroup sums the per-row losses");
static_assert(kMaxK <= 48, "three 16-row blocks of output channels");

// packed parameter offsets (floats): W1 (128 x 3), b1, W2 (128 x 128), b2, W3 (k x 128), b3
constexpr int64_t kOffB1 = 3 * kH;
constexpr int64_t kOffW2 = kOffB1 + kH;
constexpr int64_t kOffB2 = kOffW2 + kH * kH;
constexpr int64_t kOffW3 = kOffB2 + kH;
__host__ __device__ constexpr int64_t off_b3(int k) { return kOffW3 + int64_t(k) * kH; }
__host__ __device__ constexpr int64_t param_count(int k) { return off_b3(k) + k; }

typedef float f4v __attribute__((ext_vector_type(4)));

struct TrainArgs {
    int k;
    const float* params;
    const float* rgb;
    int64_t ld_rgb;
    const float* zgt;
    int64_t ld_z;
    int64_t rows;
    const uint32_t* idx;
    // rows drawn on the device: counter base draw_ctr0 (+ *draw_scale * N)
    int draw;
    uint64_t key, draw_ctr0;
    const int64_t* draw_scale;
    int64_t N;
    const float* M;  // 3 x k
    float wx, wy, wz;  // reference white
    float w_max, w_col;
    float* part;     // gridDim.x rows of P floats
    double* loss_part;
};

__device__ __forceinline__ float logistic(float x) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
    const float s = __builtin_amdgcn_rcpf(1.0f + e);
    return x >= 0.f ? s : e * s;
}

// d silu / dx = s + x s (1 - s), s = logistic(x)
__device__ __forceinline__ float dsilu(float x) {
    const float sg = logistic(x);
    return sg + x * sg * (1.f - sg);
}

__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS row strides and layout of the partials kernel.  Activations are
// [feature][sample] arrays with 17 floats per feature row and 16 more after
// every 32 rows, so the MFMA operand reads of both orientations (16 samples
// of 4 rows, 16 rows 32 apart, 16 rows of 4 samples) fall on distinct banks.
__device__ __forceinline__ int act(int r, int s) { return r * kAS + (r >> 5) * 16 + s; }
constexpr int kActSize = kH * kAS + (kH / 32) * 16;
static_assert(kPWaves * 8 * kRS <= 4 * kActSize, "W2 staging slices fit in P1..H2");

struct Lds {
    float *W3, *W1, *B2, *B3, *M, *X, *P1, *H1, *P2, *H2, *Z, *G, *ZP, *S;
    double* loss;
};

__device__ __forceinline__ Lds lds_areas(float* sm, int k) {
    Lds L;
    L.W3 = sm;                        // k x kRS
    L.W1 = L.W3 + k * kRS;            // 128 x 4: (w_r, w_g, w_b, b1), the A operand of layer 1
    L.B2 = L.W1 + 4 * kH;
    L.B3 = L.B2 + kH;                 // 48
    L.M = L.B3 + kMaxK;               // 3 x 48
    L.X = L.M + 3 * kMaxK;            // 16 samples x (r, g, b, 1)
    L.P1 = L.X + 4 * kTS;             // p1, then dL/dp1
    L.H1 = L.P1 + kActSize;
    L.P2 = L.H1 + kActSize;           // p2, then dL/dp2
    L.H2 = L.P2 + kActSize;
    L.Z = L.H2 + kActSize;            // 48 x kAS: z
    L.G = L.Z + kMaxK * kAS;          // 48 x kAS: target code, then dL/dz (rows k..47 zero)
    L.ZP = L.G + kMaxK * kAS;         // layer-3 partial products: 8 waves x 3 blocks x 256
    L.S = L.ZP + kPWaves * 3 * 256;   // per sample: channel of the max-abs term, colour gradient (4 x 16)
    L.loss = reinterpret_cast<double*>(L.S + 4 * kTS);   // an even float offset: 8-byte aligned
    return L;
}

size_t lds_bytes(int k) {
    return sizeof(float) * (size_t(k) * kRS + 4 * kH + kH + kMaxK + 3 * kMaxK + 4 * kTS + 4 * size_t(kActSize) +
                            2 * size_t(kMaxK) * kAS + kPWaves * 3 * 256 + 4 * kTS) +
           sizeof(double) * kTS;
}

// cube root of t > 0 from the hardware base-2 logarithm and exponential
__device__ __forceinline__ float cbrt_pos(float t) {
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(t) * (1.0f / 3.0f));
}

// CIELAB f and its slope
__device__ __forceinline__ void lab_f(float t, float& f, float& fp) {
    constexpr float d = 6.0f / 29.0f;
    if (t > d * d * d) {
        const float c = cbrt_pos(t);
        f = c;
        fp = 1.0f / (3.0f * c * c);
    } else {
        f = t / (3.0f * d * d) + 4.0f / 29.0f;
        fp = 1.0f / (3.0f * d * d);
    }
}

// One workgroup per partial row; it takes tiles of 16 samples in turn.  Per
// tile, with the activations of the tile in LDS as [feature][sample]:
//   forward   p1 = W1 c + b1 (one 16x16x4 product per 16 features, the bias
//             through a constant-1 input), p2 = W2 h1 + b2 (32 products per
//             16 features, W2's fragments held in registers), z = W3 h2 + b3
//             (the 128-long sums split over the 8 wavefronts, then added in
//             a fixed order);
//   loss      per sample: the three terms of Sec. 5.2 and dL/dz;
//   backward  dL/dh2 = W3^T dL/dz, dL/dp2 = dL/dh2 * silu'(p2), dL/dh1 =
//             W2^T dL/dp2, dL/dp1 = dL/dh1 * silu'(p1) (matrix cores), and the
//             weight gradients dW3 += dz h2^T, dW2 += dp2 h1^T, [dW1 db1] +=
//             dp1 [c 1]^T as 16x16x4 products over the tile's samples,
//             accumulated in registers across tiles; bias sums on the ALU.
// Samples past N have dL/dz = 0, so they add nothing.
__global__ __launch_bounds__(kPThreads) void ustrain_partials_kernel(TrainArgs a) {
    extern __shared__ __align__(16) float sm[];
    const int k = a.k;
    const Lds L = lds_areas(sm, k);
    const int tid = threadIdx.x;
    const int w = tid / 64, lane = tid & 63, g = lane / 16, n = lane % 16;
    const int jrow = 16 * w;           // the wave's 16 hidden rows
    const float* P = a.params;
    const int mc3 = (k + 15) / 16;         // 16-row blocks of output channels
    const int ksteps = (k + 3) / 4;        // K steps over the channels
    const uint64_t ctr_base =
        a.draw ? a.draw_ctr0 + (a.draw_scale ? uint64_t(*a.draw_scale) * uint64_t(a.N) : 0ull) : 0ull;
    const int64_t tiles = (a.N + kTS - 1) / kTS;

    // Loads are issued in this order: W2 (most of the bytes), the parameters
    // staged in LDS, then the first tile's inputs, whose row indices wait for
    // the step counter's load.  Each wave holds W2 fragments for the whole
    // kernel, K index 32 g + st: the forward A operand W2[jrow + n][32 g + st]
    // in wf and the backward one W2[32 g + st][jrow + n] in wb.  A lane's wf
    // values are 32 consecutive floats of one row, but the lanes of a load
    // would span 64 rows and chunks; so (parameters 16-byte aligned) the
    // wave's 16 rows are loaded whole, 1 KB per load, and handed to the lanes
    // through the wave's own slice of the activation arrays below.
    const bool al16 = (reinterpret_cast<uintptr_t>(P) & 15) == 0;
    float wf[32], wb[32];
    float4 rows4[8];   // rows jrow + 2u and jrow + 2u + 1 of W2, 4 floats a lane
    if (al16) {
#pragma unroll
        for (int u = 0; u < 8; ++u) rows4[u] = ld4(P + kOffW2 + (jrow + 2 * u) * kH + 4 * lane);
    } else {
#pragma unroll
        for (int st = 0; st < 32; ++st) wf[st] = ldg_f32(P + kOffW2 + (jrow + n) * kH + 32 * g + st);
    }
#pragma unroll
    for (int st = 0; st < 32; ++st) wb[st] = ldg_f32(P + kOffW2 + (32 * g + st) * kH + jrow + n);
    constexpr int kW3Per = (kMaxK * kH + kPThreads - 1) / kPThreads;
    float w3v[kW3Per];
#pragma unroll
    for (int u = 0; u < kW3Per; ++u) {
        const int e = tid + u * kPThreads;
        w3v[u] = e < k * kH ? P[kOffW3 + e] : 0.f;
    }
    float w1v[4] = {0.f, 0.f, 0.f, 0.f}, b2v = 0.f;
    if (tid < kH) {
        w1v[0] = P[3 * tid];
        w1v[1] = P[3 * tid + 1];
        w1v[2] = P[3 * tid + 2];
        w1v[3] = P[kOffB1 + tid];
        b2v = P[kOffB2 + tid];
    }
    const float b3v = tid < kMaxK && tid < k ? P[off_b3(k) + tid] : 0.f;
    const float mv = tid < 3 * kMaxK && (tid % kMaxK) < k ? a.M[(tid / kMaxK) * k + tid % kMaxK] : 0.f;
    // a tile's inputs: item e < kTS (k + 1) of thread tid is (sample e % 16,
    // channel e / 16 - 1), channel -1 being the colour (r, g, b, 1)
    constexpr int kInPer = (kTS * (kMaxK + 1) + kPThreads - 1) / kPThreads;
    float inv[kInPer][4];
    auto fetch_inputs = [&](int64_t tile) {
#pragma unroll
        for (int u = 0; u < kInPer; ++u) {
            const int e = tid + u * kPThreads;
            inv[u][0] = inv[u][1] = inv[u][2] = inv[u][3] = 0.f;
            if (e < kTS * (k + 1)) {
                const int i = e % kTS, c = e / kTS - 1;
                const int64_t s = tile * kTS + i;
                if (s < a.N) {
                    const int64_t row =
                        a.draw ? int64_t(range32(rand64(a.key, ctr_base + uint64_t(s)), uint64_t(a.rows)))
                               : (a.idx ? min<int64_t>(a.idx[s], a.rows - 1) : s);
                    if (c < 0) {
                        const float* cp = a.rgb + row * a.ld_rgb;
                        inv[u][0] = cp[0];
                        inv[u][1] = cp[1];
                        inv[u][2] = cp[2];
                        inv[u][3] = 1.f;
                    } else {
                        inv[u][0] = a.zgt[row * a.ld_z + 4 * (c / 3) + c % 3];
                    }
                }
            }
        }
    };
    auto store_inputs = [&]() {
#pragma unroll
        for (int u = 0; u < kInPer; ++u) {
            const int e = tid + u * kPThreads;
            if (e < kTS * (k + 1)) {
                const int i = e % kTS, c = e / kTS - 1;
                if (c < 0) {
                    L.X[4 * i + 0] = inv[u][0];
                    L.X[4 * i + 1] = inv[u][1];
                    L.X[4 * i + 2] = inv[u][2];
                    L.X[4 * i + 3] = inv[u][3];
                } else {
                    L.G[c * kAS + i] = inv[u][0];
                }
            }
        }
    };
    fetch_inputs(blockIdx.x);
    if (al16) {
        // wf from the staged rows, 8 rows a pass, in the wave's own 8 x kRS
        // floats of P1..H2 (not in use before the first tile's layer 1; the
        // wave's LDS accesses complete in order, so pass 1 may overwrite
        // what pass 0 read)
        float* stg = L.P1 + w * (8 * kRS);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                *reinterpret_cast<float4*>(stg + (2 * u + lane / 32) * kRS + 4 * (lane % 32)) = rows4[4 * h + u];
            if ((n >> 3) == h) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float4 v = *reinterpret_cast<const float4*>(stg + (n - 8 * h) * kRS + 32 * g + 4 * q);
                    wf[4 * q] = v.x;
                    wf[4 * q + 1] = v.y;
                    wf[4 * q + 2] = v.z;
                    wf[4 * q + 3] = v.w;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kW3Per; ++u) {
        const int e = tid + u * kPThreads;
        if (e < k * kH) L.W3[(e / kH) * kRS + e % kH] = w3v[u];
    }
    if (tid < kH) {
        L.W1[4 * tid + 0] = w1v[0];
        L.W1[4 * tid + 1] = w1v[1];
        L.W1[4 * tid + 2] = w1v[2];
        L.W1[4 * tid + 3] = w1v[3];
        L.B2[tid] = b2v;
    }
    if (tid < kMaxK) L.B3[tid] = b3v;
    if (tid < 3 * kMaxK) L.M[tid] = mv;
    // rows k..47 of the code arrays stay zero for every tile
    for (int e = tid; e < 2 * kMaxK * kAS; e += kPThreads) L.Z[e] = 0.f;

    f4v acc2[8], acc3[3], acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 8; ++b) acc2[b] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 3; ++b) acc3[b] = f4v{0.f, 0.f, 0.f, 0.f};
    float aB2 = 0.f, aB3 = 0.f;
    double loss = 0.0;
    __syncthreads();

    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        // ---- inputs of the tile: colours (+ the constant 1) and target codes
        if (tile != blockIdx.x) fetch_inputs(tile);
        store_inputs();
        __syncthreads();
        // ---- layer 1 (K = 4: r, g, b, 1)
        {
            const f4v d = mfma4(L.W1[4 * (jrow + n) + g], L.X[4 * n + g], f4v{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jrow + 4 * g + r;
                L.P1[act(j, n)] = d[r];
                L.H1[act(j, n)] = d[r] * logistic(d[r]);
            }
        }
        __syncthreads();
        // ---- layer 2: 32 K steps, two independent chains
        {
            f4v c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 32; st += 2) {
                c0 = mfma4(wf[st], L.H1[act(32 * g + st, n)], c0);
                c1 = mfma4(wf[st + 1], L.H1[act(32 * g + st + 1, n)], c1);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jrow + 4 * g + r;
                const float v = (c0[r] + c1[r]) + L.B2[j];
                L.P2[act(j, n)] = v;
                L.H2[act(j, n)] = v * logistic(v);
            }
        }
        __syncthreads();
        // ---- layer 3: wave w sums hidden rows 16w..16w+15 for every block of
        // channels; the eight partial products are added in order below
        {
#pragma unroll
            for (int mc = 0; mc < 3; ++mc) {
                if (mc < mc3) {
                    const int c = 16 * mc + n;
                    f4v d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        const int i = jrow + 4 * st + g;
                        d = mfma4(c < k ? L.W3[c * kRS + i] : 0.f, L.H2[act(i, n)], d);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) L.ZP[(w * 3 + mc) * 256 + (4 * g + r) * 16 + n] = d[r];
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < k * kTS; e += kPThreads) {
            const int c = e / kTS, i = e % kTS, mc = c / 16, cr = c % 16;
            float v = 0.f;
#pragma unroll
            for (int ww = 0; ww < kPWaves; ++ww) v += L.ZP[(ww * 3 + mc) * 256 + cr * 16 + i];
            L.Z[c * kAS + i] = v + L.B3[c];
        }
        __syncthreads();
        // ---- per-sample loss terms and the colour gradient: lanes i, i + 16 and
        // i + 32 of wavefront 0 take sample i's X, Y and Z (and its CIELAB f),
        // exchange the three f values, and each forms the rest of the sample's
        // terms; the lane of X also sums the code terms
        if (tid < 3 * kTS) {
            const int i = tid % kTS, x = tid / kTS;
            const bool valid = tile * kTS + i < a.N;
            const float wh = x == 0 ? a.wx : (x == 1 ? a.wy : a.wz);
            float Xx = 0.f, Xgx = 0.f;
            for (int c = 0; c < k; ++c) {
                Xx = fmaf(L.M[x * kMaxK + c], L.Z[c * kAS + i], Xx);
                Xgx = fmaf(L.M[x * kMaxK + c], L.G[c * kAS + i], Xgx);
            }
            float f, fp, fg, unused;
            lab_f(Xx / wh, f, fp);
            lab_f(Xgx / wh, fg, unused);
            const float f0 = __shfl(f, i, kWave), f1 = __shfl(f, i + kTS, kWave), f2 = __shfl(f, i + 2 * kTS, kWave);
            const float g0 = __shfl(fg, i, kWave), g1 = __shfl(fg, i + kTS, kWave),
                        g2 = __shfl(fg, i + 2 * kTS, kWave);
            const float dL = 116.f * (f1 - g1);
            const float da = 500.f * ((f0 - f1) - (g0 - g1));
            const float db = 200.f * ((f1 - f2) - (g1 - g2));
            const float de = sqrtf(dL * dL + da * da + db * db);
            const float inv = de > 0.f ? 1.f / de : 0.f;
            const float uL = dL * inv, ua = da * inv, ub = db * inv;
            // gradient of DeltaE76 with respect to the predicted XYZ
            const float gx = x == 0 ? 500.f * ua : (x == 1 ? 116.f * uL - 500.f * ua + 200.f * ub : -200.f * ub);
            L.S[(1 + x) * kTS + i] = gx * fp / wh;
            if (x == 0) {
                float mse = 0.f, amax = -1.f;
                int cs = 0;
                for (int c = 0; c < k; ++c) {
                    const float d = L.Z[c * kAS + i] - L.G[c * kAS + i];
                    mse = fmaf(d, d, mse);
                    if (fabsf(d) > amax) {      // the first channel of largest |d|
                        amax = fabsf(d);
                        cs = c;
                    }
                }
                L.S[i] = valid ? __int_as_float(cs) : __int_as_float(-1);
                if (valid) loss += double(mse) / k + double(a.w_max) * amax + double(a.w_col) * de;
            }
        }
        __syncthreads();
        // ---- dL/dz (one thread per channel and sample), in place of the target
        for (int e = tid; e < k * kTS; e += kPThreads) {
            const int c = e / kTS, i = e % kTS;
            const int cs = __float_as_int(L.S[i]);
            const float d = L.Z[c * kAS + i] - L.G[c * kAS + i];
            float gz = (2.0f / k) * d;
            if (c == cs) gz += a.w_max * (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f));
            gz += a.w_col * (L.M[c] * L.S[kTS + i] + L.M[kMaxK + c] * L.S[2 * kTS + i] +
                             L.M[2 * kMaxK + c] * L.S[3 * kTS + i]);
            L.G[c * kAS + i] = cs >= 0 ? gz : 0.f;       // cs < 0: a sample past N
        }
        __syncthreads();
        // ---- dL/dp2 (in place of p2), dW3 += dz h2^T, db3
        {
            f4v d = {0.f, 0.f, 0.f, 0.f};
            for (int st = 0; st < ksteps; ++st) {
                const int c = 4 * st + g;
                d = mfma4(c < k ? L.W3[c * kRS + jrow + n] : 0.f, L.G[c * kAS + n], d);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jrow + 4 * g + r;
                L.P2[act(j, n)] = d[r] * dsilu(L.P2[act(j, n)]);
            }
#pragma unroll
            for (int mc = 0; mc < 3; ++mc) {
                if (mc < mc3) {
#pragma unroll
                    for (int st = 0; st < kTS / 4; ++st)
                        acc3[mc] = mfma4(L.G[(16 * mc + n) * kAS + 4 * st + g], L.H2[act(jrow + n, 4 * st + g)],
                                         acc3[mc]);
                }
            }
            if (tid < k) {
                float t = 0.f;
                for (int i = 0; i < kTS; ++i) t += L.G[tid * kAS + i];
                aB3 += t;
            }
        }
        __syncthreads();
        // ---- dL/dp1 (in place of p1), dW2 += dp2 h1^T, db2
        {
            f4v c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 32; st += 2) {
                c0 = mfma4(wb[st], L.P2[act(32 * g + st, n)], c0);
                c1 = mfma4(wb[st + 1], L.P2[act(32 * g + st + 1, n)], c1);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jrow + 4 * g + r;
                L.P1[act(j, n)] = (c0[r] + c1[r]) * dsilu(L.P1[act(j, n)]);
            }
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
#pragma unroll
                for (int st = 0; st < kTS / 4; ++st)
                    acc2[nb] = mfma4(L.P2[act(jrow + n, 4 * st + g)], L.H1[act(16 * nb + n, 4 * st + g)], acc2[nb]);
            }
            if (tid < kH) {
                float t = 0.f;
                for (int i = 0; i < kTS; ++i) t += L.P2[act(tid, i)];
                aB2 += t;
            }
        }
        __syncthreads();
        // ---- [dW1 db1] += dp1 [c 1]^T
#pragma unroll
        for (int st = 0; st < kTS / 4; ++st)
            acc1 = mfma4(L.P1[act(jrow + n, 4 * st + g)], n < 4 ? L.X[4 * (4 * st + g) + n] : 0.f, acc1);
        __syncthreads();
    }
    // workgroup loss: the per-sample lanes 0..15, in order (before the row's stores,
    // so that no barrier waits for them)
    if (tid < kTS) L.loss[tid] = loss;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < kTS; ++i) t += L.loss[i];
        a.loss_part[blockIdx.x] = t;
    }
    // ---- partial row, with non-temporal stores (read once, by kernel 2)
    float* prow = a.part + int64_t(blockIdx.x) * param_count(k);
#pragma unroll
    for (int nb = 0; nb < 8; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) __builtin_nontemporal_store(acc2[nb][r], &prow[kOffW2 + (jrow + 4 * g + r) * kH + 16 * nb + n]);
#pragma unroll
    for (int mc = 0; mc < 3; ++mc)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * mc + 4 * g + r;
            if (mc < mc3 && c < k) __builtin_nontemporal_store(acc3[mc][r], &prow[kOffW3 + c * kH + jrow + n]);
        }
    if (n < 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = jrow + 4 * g + r;
            __builtin_nontemporal_store(acc1[r], &prow[n < 3 ? 3 * j + n : kOffB1 + j]);
        }
    }
    if (tid < kH) __builtin_nontemporal_store(aB2, &prow[kOffB2 + tid]);
    if (tid < k) __builtin_nontemporal_store(aB3, &prow[off_b3(k) + tid]);
}

struct ReduceArgs {
    int64_t P, N;
    int rows;
    const float* part;
    const double* loss_part;
    float* grad;
    double* sq_part;  // per block
    float* loss;
    int64_t* step;     // nullable: bumped once
    int64_t* ws_step;
};

// Sum of x[0 .. count) by the calling workgroup, in a fixed order: thread t
// adds x[t], x[t + 256], ... (thread_terms, issued early so that its loads
// overlap the kernel's other loads), then block_sum adds those with a
// butterfly inside each wavefront, then the wavefronts in order.  The result
// is valid in thread 0.
__device__ __forceinline__ double thread_terms(const double* x, int count) {
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += kThreads) v += x[i];
    return v;
}

__device__ double block_sum(double v) {
    __shared__ double s_w[kThreads / kWave];
    for (int m = kWave / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / kWave; ++w) t += s_w[w];
    return t;
}

// A block reduces 64 parameters: its four wavefronts sum a quarter of the
// partial rows each (sixteen row loads in flight per lane), then the quarters
// are added in order.
constexpr int kRedParams = kWave;
constexpr int kRedQuarters = kThreads / kWave;

__global__ __launch_bounds__(kThreads) void ustrain_reduce_kernel(ReduceArgs a) {
    const int q = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t e = int64_t(blockIdx.x) * kRedParams + lane;
    const int per = (a.rows + kRedQuarters - 1) / kRedQuarters;
    const int r0 = min(a.rows, q * per), r1 = min(a.rows, r0 + per);
    __shared__ double s_part[kRedQuarters][kRedParams];
    // block 0's share of the loss sum and the step counter, read first
    const double loss_terms = blockIdx.x == 0 ? thread_terms(a.loss_part, a.rows) : 0.0;
    const int64_t step0 = blockIdx.x == 0 && a.step ? *a.step : 0;
    double part = 0.0;
    if (e < a.P) {
        // sixteen interleaved partial sums keep sixteen row loads in flight
        // (whole batches unguarded: a guarded load becomes a branch per row)
        constexpr int kIlp = 16;
        double acc[kIlp];
#pragma unroll
        for (int u = 0; u < kIlp; ++u) acc[u] = 0.0;
        int r = r0;
        for (; r + kIlp <= r1; r += kIlp) {
            float x[kIlp];
#pragma unroll
            for (int u = 0; u < kIlp; ++u) x[u] = a.part[int64_t(r + u) * a.P + e];
#pragma unroll
            for (int u = 0; u < kIlp; ++u) acc[u] += double(x[u]);
        }
        for (; r < r1; ++r) acc[0] += double(a.part[int64_t(r) * a.P + e]);
#pragma unroll
        for (int w = kIlp / 2; w >= 1; w >>= 1)
#pragma unroll
            for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
        part = acc[0];
    }
    s_part[q][lane] = part;
    __syncthreads();
    double sq = 0.0;
    if (q == 0) {
        double g = 0.0;
        if (e < a.P) {
#pragma unroll
            for (int u = 0; u < kRedQuarters; ++u) g += s_part[u][lane];
            g /= double(a.N);
            a.grad[e] = float(g);
        }
        sq = g * g;
        for (int m = kWave / 2; m >= 1; m >>= 1) sq += __shfl_xor(sq, m, kWave);
        if (lane == 0) a.sq_part[blockIdx.x] = sq;
    }
    if (blockIdx.x == 0) {
        const double l = block_sum(loss_terms);
        if (threadIdx.x == 0) {
            *a.loss = float(l / double(a.N));
            if (a.step) {
                const int64_t t1 = step0 + 1;
                *a.ws_step = t1;
                *a.step = t1;
            }
        }
    }
}

struct AdamWArgs {
    int64_t P;
    int nsq;
    const double* sq_part;
    const float* grad;
    float* params;
    float* m;
    float* v;
    const int64_t* ws_step;
    double lr, beta1, beta2, eps, wd, max_norm;
    double ln_beta1, ln_beta2;
};

__global__ __launch_bounds__(kThreads) void ustrain_adamw_kernel(AdamWArgs a) {
    __shared__ double s_c[3];
    // the parameter's operands and the step counter are loaded with the
    // block sums, in one round of loads
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const bool live = e < a.P;
    float g0 = 0.f, w0 = 0.f, m0 = 0.f, v0 = 0.f;
    if (live) {
        g0 = a.grad[e];
        w0 = a.params[e];
        m0 = a.m[e];
        v0 = a.v[e];
    }
    const int64_t step = *a.ws_step;
    // every block forms the same norm from the block sums, and the step's
    // bias corrections (beta^t = exp(t ln beta), ln beta from the host)
    const double t2 = block_sum(thread_terms(a.sq_part, a.nsq));
    if (threadIdx.x == 0) {
        const double norm = sqrt(t2);
        const double c = a.max_norm / (norm + 1e-6);
        const double t = double(step);
        s_c[0] = c < 1.0 ? c : 1.0;
        s_c[1] = a.lr / (1.0 - exp(t * a.ln_beta1));
        s_c[2] = 1.0 / sqrt(1.0 - exp(t * a.ln_beta2));
    }
    __syncthreads();
    if (!live) return;
    const double g = double(g0) * s_c[0];
    const double w = double(w0) * (1.0 - a.lr * a.wd);
    const double mm = a.beta1 * double(m0) + (1.0 - a.beta1) * g;
    const double vv = a.beta2 * double(v0) + (1.0 - a.beta2) * g * g;
    a.m[e] = float(mm);
    a.v[e] = float(vv);
    a.params[e] = float(w - s_c[1] * mm / (sqrt(vv) * s_c[2] + a.eps));
}

int64_t grid_rows(int64_t N) { return std::min<int64_t>((N + kTS - 1) / kTS, kMaxRows); }


size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Ws {
    float* part;
    double* loss_part;
    double* sq_part;
    float* grad;
    int64_t* step;
};

Ws carve(void* base, int k, int64_t N) {
    const int64_t P = param_count(k);
    const int64_t rows = grid_rows(N);
    const int64_t nsq = ceil_div(P, kRedParams);
    char* p = static_cast<char*>(base);
    Ws w;
    w.part = reinterpret_cast<float*>(p);
    p += align256(size_t(rows) * P * sizeof(float));
    w.loss_part = reinterpret_cast<double*>(p);
    p += align256(size_t(kMaxRows) * sizeof(double));
    w.sq_part = reinterpret_cast<double*>(p);
    p += align256(size_t(nsq) * sizeof(double));
    w.grad = reinterpret_cast<float*>(p);
    p += align256(size_t(P) * sizeof(float));
    w.step = reinterpret_cast<int64_t*>(p);
    return w;
}

}  // namespace

int64_t upsample_param_count(int k) { return param_count(k); }

size_t upsample_train_workspace_size(int k, int64_t N) {
    const int64_t P = param_count(k);
    return align256(size_t(grid_rows(N)) * P * sizeof(float)) + align256(kMaxRows * sizeof(double)) +
           align256(size_t(ceil_div(P, kRedParams)) * sizeof(double)) + align256(size_t(P) * sizeof(float)) +
           sizeof(int64_t);
}

hc_status launch_upsample_train(const hc_upsample_train_args& u) {
    hipStream_t st = reinterpret_cast<hipStream_t>(u.stream);
    const int k = u.k;
    const int64_t P = param_count(k);
    const int64_t rows = grid_rows(u.N);
    Ws ws = carve(u.workspace, k, u.N);
    TrainArgs a;
    a.k = k;
    a.params = u.params;
    a.rgb = u.rgb;
    a.ld_rgb = u.ld_rgb;
    a.zgt = u.z_gt;
    a.ld_z = u.ld_z;
    a.rows = u.rows;
    a.idx = u.idx;
    a.draw = u.draw != nullptr;
    a.key = u.draw ? stream_key(u.draw->seed, kIndexStream) : 0;
    a.draw_ctr0 = u.draw ? u.draw->ctr0 : 0;
    a.draw_scale = u.draw ? u.draw->ctr_scale_dev : nullptr;
    a.N = u.N;
    a.M = u.M;
    a.wx = float(u.white[0]);
    a.wy = float(u.white[1]);
    a.wz = float(u.white[2]);
    a.w_max = float(u.w_max);
    a.w_col = float(u.w_col);
    a.part = ws.part;
    a.loss_part = ws.loss_part;
    hipLaunchKernelGGL(ustrain_partials_kernel, dim3(uint32_t(rows)), dim3(kPThreads), lds_bytes(k), st, a);
    hc_status s = launch_status("hc_upsample_train_step");
    if (s != HC_OK) return s;

    ReduceArgs r;
    r.P = P;
    r.N = u.N;
    r.rows = int(rows);
    r.part = ws.part;
    r.loss_part = ws.loss_part;
    r.grad = u.grad ? u.grad : ws.grad;
    r.sq_part = ws.sq_part;
    r.loss = u.loss;
    r.step = u.opt ? u.opt->step : nullptr;
    r.ws_step = ws.step;
    const int nsq = int(ceil_div(P, kRedParams));
    hipLaunchKernelGGL(ustrain_reduce_kernel, dim3(nsq), dim3(kThreads), 0, st, r);
    s = launch_status("hc_upsample_train_step");
    if (s != HC_OK || !u.opt) return s;

    AdamWArgs w;
    w.P = P;
    w.nsq = nsq;
    w.sq_part = ws.sq_part;
    w.grad = r.grad;
    w.params = u.params;
    w.m = u.opt->m;
    w.v = u.opt->v;
    w.ws_step = ws.step;
    w.lr = u.opt->lr;
    w.beta1 = u.opt->beta1;
    w.beta2 = u.opt->beta2;
    // beta = 0 gives exp(t * -inf) = 0 for every step t >= 1
    w.ln_beta1 = std::log(u.opt->beta1);
    w.ln_beta2 = std::log(u.opt->beta2);
    w.eps = u.opt->eps;
    w.wd = u.opt->weight_decay;
    w.max_norm = u.opt->max_grad_norm;
    hipLaunchKernelGGL(ustrain_adamw_kernel, dim3(int(ceil_div(P, kThreads))), dim3(kThreads), 0, st, w);
    return launch_status("hc_upsample_train_step");
}

}  // namespace hc
