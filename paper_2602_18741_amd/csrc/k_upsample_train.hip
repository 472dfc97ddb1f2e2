// Training step of the upsampling network (Sec. 5.2): loss, hand-written
// backward and AdamW with global-norm gradient clipping, on a batch of
// (RGB, code) pairs gathered by index or drawn from the counter-based
// generator inside kernel 1.  Deterministic: fixed summation orders, no
// floating-point atomics.
//
//   1. partials: a workgroup (at most one per CU's worth: 256 partial rows)
//                takes four samples at a time, one per quarter (128 threads,
//                one per hidden unit).  Forward through the
//                three layers, the per-sample loss terms and dL/dz, then
//                backward to the hidden pre-activations, with W2 and W3 in LDS
//                (odd row stride: row-wise and column-wise reads are both
//                conflict-free).  Every thread owns a fixed set of gradient
//                elements and accumulates them over the workgroup's samples
//                in registers; one partial row per workgroup.
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
constexpr int kThreads = 256;
constexpr int kSamples = 4;        // samples a partials workgroup takes at once
constexpr int kPThreads = kSamples * kH;
// LDS row stride of W2 and W3: rows 16-byte aligned for the forward's row
// reads, 4 banks apart so 16 threads' rows and a row's columns are spread
constexpr int kRS = kH + 4;
constexpr int kMaxRows = 256;      // partial rows (workgroups of kernel 1): one per CU
static_assert(kMaxRows <= kThreads, "one workgroup sums the per-row losses");
constexpr int kW3PerThread = kMaxK / kSamples;
constexpr int kW2PerThread = kH / kSamples;
static_assert(kRS % 4 == 0 && (6 * kH + 3 * kMaxK + 8) % 4 == 0 && kMaxK % 4 == 0,
              "16-byte aligned rows and per-sample areas in LDS");

// packed parameter offsets (floats): W1 (128 x 3), b1, W2 (128 x 128), b2, W3 (k x 128), b3
constexpr int64_t kOffB1 = 3 * kH;
constexpr int64_t kOffW2 = kOffB1 + kH;
constexpr int64_t kOffB2 = kOffW2 + kH * kH;
constexpr int64_t kOffW3 = kOffB2 + kH;
__host__ __device__ constexpr int64_t off_b3(int k) { return kOffW3 + int64_t(k) * kH; }
__host__ __device__ constexpr int64_t param_count(int k) { return off_b3(k) + k; }

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

// CIELAB f and its slope
__device__ __forceinline__ void lab_f(float t, float& f, float& fp) {
    constexpr float d = 6.0f / 29.0f;
    if (t > d * d * d) {
        const float c = cbrtf(t);
        f = c;
        fp = 1.0f / (3.0f * c * c);
    } else {
        f = t / (3.0f * d * d) + 4.0f / 29.0f;
        fp = 1.0f / (3.0f * d * d);
    }
}

__global__ __launch_bounds__(kPThreads) void ustrain_partials_kernel(TrainArgs a) {
    extern __shared__ __align__(16) float sm[];
    const int k = a.k;
    float* sW2 = sm;                    // 128 x kRS
    float* sW3 = sW2 + kH * kRS;        // k x kRS
    float* sW1 = sW3 + k * kRS;         // 128 x 4 (w_r, w_g, w_b, b1)
    float* sB2 = sW1 + 4 * kH;
    float* sB3 = sB2 + kH;              // k
    float* sM = sB3 + kMaxK;            // 3 x k
    float* sS = sM + 3 * kMaxK;         // per sample: p1, h1, p2, h2, dp2, dp1 (128 each), z, d, dz (48 each), misc 8
    constexpr int kPer = 6 * kH + 3 * kMaxK + 8;

    const int tid = threadIdx.x;
    const float* P = a.params;
    for (int e = tid; e < kH * kH; e += kPThreads) sW2[(e / kH) * kRS + e % kH] = P[kOffW2 + e];
    for (int e = tid; e < k * kH; e += kPThreads) sW3[(e / kH) * kRS + e % kH] = P[kOffW3 + e];
    for (int j = tid; j < kH; j += kPThreads) {
        sW1[4 * j + 0] = P[3 * j];
        sW1[4 * j + 1] = P[3 * j + 1];
        sW1[4 * j + 2] = P[3 * j + 2];
        sW1[4 * j + 3] = P[kOffB1 + j];
        sB2[j] = P[kOffB2 + j];
    }
    for (int c = tid; c < k; c += kPThreads) sB3[c] = P[off_b3(k) + c];
    for (int e = tid; e < 3 * k; e += kPThreads) sM[e] = a.M[e];

    const int smp = tid / kH, j = tid % kH;  // the thread's sample of the four, hidden unit
    float* S = sS + smp * kPer;
    float* p1 = S;
    float* h1 = p1 + kH;
    float* p2 = h1 + kH;
    float* h2 = p2 + kH;
    float* dp2 = h2 + kH;
    float* dp1 = dp2 + kH;
    float* zz = dp1 + kH;
    float* dd = zz + kMaxK;
    float* dz = dd + kMaxK;
    float* misc = dz + kMaxK;  // rgb (3), gX (3)

    // gradient elements owned by this thread
    float aW2[kW2PerThread];
#pragma unroll
    for (int q = 0; q < kW2PerThread; ++q) aW2[q] = 0.f;
    float aW3[kW3PerThread];
#pragma unroll
    for (int r = 0; r < kW3PerThread; ++r) aW3[r] = 0.f;
    float aB = 0.f, aW1[3] = {0.f, 0.f, 0.f}, aB3 = 0.f;
    double loss = 0.0;
    __syncthreads();

    const uint64_t ctr_base =
        a.draw ? a.draw_ctr0 + (a.draw_scale ? uint64_t(*a.draw_scale) * uint64_t(a.N) : 0ull) : 0ull;
    const int64_t groups = (a.N + kSamples - 1) / kSamples;
    for (int64_t pr = blockIdx.x; pr < groups; pr += gridDim.x) {
        const int64_t s = kSamples * pr + smp;
        const bool valid = s < a.N;
        int64_t row = 0;
        if (valid)
            row = a.draw ? int64_t(range32(rand64(a.key, ctr_base + uint64_t(s)), uint64_t(a.rows)))
                         : (a.idx ? min<int64_t>(a.idx[s], a.rows - 1) : s);
        // forward
        const float* cp = a.rgb + row * a.ld_rgb;
        const float cr = valid ? cp[0] : 0.f, cg = valid ? cp[1] : 0.f, cb = valid ? cp[2] : 0.f;
        if (j == 0) {
            misc[0] = cr;
            misc[1] = cg;
            misc[2] = cb;
        }
        {
            const float v = fmaf(sW1[4 * j], cr, fmaf(sW1[4 * j + 1], cg, fmaf(sW1[4 * j + 2], cb, sW1[4 * j + 3])));
            p1[j] = v;
            h1[j] = v * logistic(v);
        }
        __syncthreads();
        {
            float v = sB2[j];
            const float4* wr = reinterpret_cast<const float4*>(sW2 + j * kRS);
            const float4* hv = reinterpret_cast<const float4*>(h1);
#pragma unroll 8
            for (int i = 0; i < kH / 4; ++i) {
                const float4 w = wr[i], x = hv[i];
                v = fmaf(w.x, x.x, v);
                v = fmaf(w.y, x.y, v);
                v = fmaf(w.z, x.z, v);
                v = fmaf(w.w, x.w, v);
            }
            p2[j] = v;
            h2[j] = v * logistic(v);
        }
        __syncthreads();
        if (j < k) {
            float v = sB3[j];
            const float4* wr = reinterpret_cast<const float4*>(sW3 + j * kRS);
            const float4* hv = reinterpret_cast<const float4*>(h2);
#pragma unroll 8
            for (int i = 0; i < kH / 4; ++i) {
                const float4 w = wr[i], x = hv[i];
                v = fmaf(w.x, x.x, v);
                v = fmaf(w.y, x.y, v);
                v = fmaf(w.z, x.z, v);
                v = fmaf(w.w, x.w, v);
            }
            const float g = valid ? a.zgt[row * a.ld_z + 4 * (j / 3) + j % 3] : v;
            zz[j] = v;
            dd[j] = v - g;
            dz[j] = g;  // the target code, until dL/dz replaces it below
        }
        __syncthreads();
        // per-sample loss terms and the colour gradient (one thread per sample)
        if (j == 0) {
            float mse = 0.f, amax = -1.f;
            int cs = 0;
            float X[3] = {0.f, 0.f, 0.f}, Xg[3] = {0.f, 0.f, 0.f};
            for (int c = 0; c < k; ++c) {
                const float d = dd[c];
                mse = fmaf(d, d, mse);
                if (fabsf(d) > amax) {
                    amax = fabsf(d);
                    cs = c;
                }
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    X[x] = fmaf(sM[x * k + c], zz[c], X[x]);
                    Xg[x] = fmaf(sM[x * k + c], dz[c], Xg[x]);
                }
            }
            const float wh[3] = {a.wx, a.wy, a.wz};
            float f[3], fp[3], fg[3], unused;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                lab_f(X[x] / wh[x], f[x], fp[x]);
                lab_f(Xg[x] / wh[x], fg[x], unused);
            }
            const float dL = 116.f * (f[1] - fg[1]);
            const float da = 500.f * ((f[0] - f[1]) - (fg[0] - fg[1]));
            const float db = 200.f * ((f[1] - f[2]) - (fg[1] - fg[2]));
            const float de = sqrtf(dL * dL + da * da + db * db);
            const float inv = de > 0.f ? 1.f / de : 0.f;
            const float uL = dL * inv, ua = da * inv, ub = db * inv;
            // gradient of DeltaE76 with respect to the predicted XYZ
            misc[3] = valid ? 500.f * ua * fp[0] / wh[0] : 0.f;
            misc[4] = valid ? (116.f * uL - 500.f * ua + 200.f * ub) * fp[1] / wh[1] : 0.f;
            misc[5] = valid ? -200.f * ub * fp[2] / wh[2] : 0.f;
            misc[6] = __int_as_float(cs);
            if (valid) loss += double(mse) / k + double(a.w_max) * amax + double(a.w_col) * de;
        }
        __syncthreads();
        if (j < k) {
            const int cs = __float_as_int(misc[6]);
            const float d = dd[j];
            float g = (2.0f / k) * d;
            if (j == cs) g += a.w_max * (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f));
            g += a.w_col * (sM[j] * misc[3] + sM[k + j] * misc[4] + sM[2 * k + j] * misc[5]);
            dz[j] = valid ? g : 0.f;
        }
        __syncthreads();
        // backward to the hidden layers
        {
            float v = 0.f;
            for (int c = 0; c < k; ++c) v = fmaf(sW3[c * kRS + j], dz[c], v);
            const float x = p2[j], sg = logistic(x);
            dp2[j] = v * (sg + x * sg * (1.f - sg));
        }
        __syncthreads();
        {
            float v = 0.f;
            for (int i = 0; i < kH; ++i) v = fmaf(sW2[i * kRS + j], dp2[i], v);
            const float x = p1[j], sg = logistic(x);
            dp1[j] = v * (sg + x * sg * (1.f - sg));
        }
        __syncthreads();
        // accumulate the four samples, in order, into the owned gradient
        // elements: W2 rows i = 32 hi + q (contiguous: 16-byte reads of dp2),
        // W3 rows c = 4r + hi, column jj
        {
            const int jj = tid % kH, hi = tid / kH;
            float h1[kSamples], h2[kSamples];
#pragma unroll
            for (int u = 0; u < kSamples; ++u) {
                h1[u] = sS[u * kPer + kH + jj];
                h2[u] = sS[u * kPer + 3 * kH + jj];
            }
#pragma unroll
            for (int q = 0; q < kW2PerThread; ++q) {
                const int i = kW2PerThread * hi + q;
                float v = aW2[q];
#pragma unroll
                for (int u = 0; u < kSamples; ++u) v = fmaf(sS[u * kPer + 4 * kH + i], h1[u], v);
                aW2[q] = v;
            }
#pragma unroll
            for (int r = 0; r < kW3PerThread; ++r) {
                const int c = kSamples * r + hi;
                if (c < k) {
                    float v = aW3[r];
#pragma unroll
                    for (int u = 0; u < kSamples; ++u) v = fmaf(sS[u * kPer + 6 * kH + 2 * kMaxK + c], h2[u], v);
                    aW3[r] = v;
                }
            }
            if (hi == 0) {
#pragma unroll
                for (int u = 0; u < kSamples; ++u) aB += sS[u * kPer + 4 * kH + jj];  // b2
            } else if (hi == 1) {
#pragma unroll
                for (int u = 0; u < kSamples; ++u) {
                    const float d1 = sS[u * kPer + 5 * kH + jj];
                    const float* mu = sS + u * kPer + 6 * kH + 3 * kMaxK;
#pragma unroll
                    for (int x = 0; x < 3; ++x) aW1[x] = fmaf(d1, mu[x], aW1[x]);
                    aB += d1;  // b1
                }
            }
            if (tid < k) {
#pragma unroll
                for (int u = 0; u < kSamples; ++u) aB3 += sS[u * kPer + 6 * kH + 2 * kMaxK + tid];
            }
        }
        __syncthreads();
    }
    // partial row
    float* prow = a.part + int64_t(blockIdx.x) * param_count(k);
    {
        const int jj = tid % kH, hi = tid / kH;
#pragma unroll
        for (int q = 0; q < kW2PerThread; ++q) prow[kOffW2 + (kW2PerThread * hi + q) * kH + jj] = aW2[q];
#pragma unroll
        for (int r = 0; r < kW3PerThread; ++r) {
            const int c = kSamples * r + hi;
            if (c < k) prow[kOffW3 + c * kH + jj] = aW3[r];
        }
        if (hi == 0) {
            prow[kOffB2 + jj] = aB;
        } else if (hi == 1) {
#pragma unroll
            for (int x = 0; x < 3; ++x) prow[3 * jj + x] = aW1[x];
            prow[kOffB1 + jj] = aB;
        }
        if (tid < k) prow[off_b3(k) + tid] = aB3;
    }
    // workgroup loss: the per-sample threads (tid 0, 128, 256, 384), fixed order
    __shared__ double s_loss[kSamples];
    if (tid % kH == 0) s_loss[tid / kH] = loss;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int u = 0; u < kSamples; ++u) t += s_loss[u];
        a.loss_part[blockIdx.x] = t;
    }
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

// Sum of x[0 .. count) (count <= kThreads) by the calling workgroup, in a fixed
// order: a butterfly inside each wavefront, then the wavefronts in order.  The
// result is valid in thread 0.
__device__ double block_sum(const double* x, int count) {
    __shared__ double s_w[kThreads / kWave];
    double v = int(threadIdx.x) < count ? x[threadIdx.x] : 0.0;
    for (int m = kWave / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / kWave; ++w) t += s_w[w];
    return t;
}

__global__ __launch_bounds__(kThreads) void ustrain_reduce_kernel(ReduceArgs a) {
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    double g = 0.0;
    if (e < a.P) {
        // sixteen interleaved partial sums keep sixteen row loads in flight
        // (whole batches unguarded: a guarded load becomes a branch per row)
        constexpr int kIlp = 16;
        double acc[kIlp];
#pragma unroll
        for (int u = 0; u < kIlp; ++u) acc[u] = 0.0;
        int r = 0;
        for (; r + kIlp <= a.rows; r += kIlp) {
            float x[kIlp];
#pragma unroll
            for (int u = 0; u < kIlp; ++u) x[u] = a.part[int64_t(r + u) * a.P + e];
#pragma unroll
            for (int u = 0; u < kIlp; ++u) acc[u] += double(x[u]);
        }
        for (; r < a.rows; ++r) acc[0] += double(a.part[int64_t(r) * a.P + e]);
#pragma unroll
        for (int w = kIlp / 2; w >= 1; w >>= 1)
#pragma unroll
            for (int u = 0; u < w; ++u) acc[u] += acc[u + w];
        g = acc[0] / double(a.N);
        a.grad[e] = float(g);
    }
    double sq = g * g;
    for (int m = kWave / 2; m >= 1; m >>= 1) sq += __shfl_xor(sq, m, kWave);
    __shared__ double s_sq[kThreads / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) s_sq[threadIdx.x / kWave] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) t += s_sq[w];
        a.sq_part[blockIdx.x] = t;
    }
    if (blockIdx.x == 0) {
        const double l = block_sum(a.loss_part, a.rows);  // rows <= kThreads
        if (threadIdx.x == 0) {
            *a.loss = float(l / double(a.N));
            if (a.step) {
                const int64_t t1 = *a.step + 1;
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
    __shared__ double s_scale;
    // every block forms the same norm from the block sums (nsq <= kThreads)
    const double t2 = block_sum(a.sq_part, a.nsq);
    if (threadIdx.x == 0) {
        const double norm = sqrt(t2);
        const double c = a.max_norm / (norm + 1e-6);
        s_scale = c < 1.0 ? c : 1.0;
    }
    __syncthreads();
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= a.P) return;
    const double g = double(a.grad[e]) * s_scale;
    const double t = double(*a.ws_step);
    const double w = double(a.params[e]) * (1.0 - a.lr * a.wd);
    const double mm = a.beta1 * double(a.m[e]) + (1.0 - a.beta1) * g;
    const double vv = a.beta2 * double(a.v[e]) + (1.0 - a.beta2) * g * g;
    // beta^t = exp(t ln beta), ln beta from the host
    const double bc1 = 1.0 - exp(t * a.ln_beta1);
    const double bc2 = 1.0 - exp(t * a.ln_beta2);
    a.m[e] = float(mm);
    a.v[e] = float(vv);
    a.params[e] = float(w - (a.lr / bc1) * mm / (sqrt(vv) / sqrt(bc2) + a.eps));
}

int64_t grid_rows(int64_t N) { return std::min<int64_t>((N + kSamples - 1) / kSamples, kMaxRows); }
static_assert((param_count(kMaxK) + kThreads - 1) / kThreads <= kThreads,
              "one workgroup sums the per-block squares");

size_t lds_bytes(int k) {
    return sizeof(float) * (size_t(kH) * kRS + size_t(k) * kRS + 4 * kH + kH + kMaxK + 3 * kMaxK +
                            kSamples * (6 * kH + 3 * kMaxK + 8));
}

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
    const int64_t nsq = ceil_div(P, kThreads);
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
           align256(size_t(ceil_div(P, kThreads)) * sizeof(double)) + align256(size_t(P) * sizeof(float)) +
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
    const int nsq = int(ceil_div(P, kThreads));
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
    hipLaunchKernelGGL(ustrain_adamw_kernel, dim3(nsq), dim3(kThreads), 0, st, w);
    return launch_status("hc_upsample_train_step");
}

}  // namespace hc
