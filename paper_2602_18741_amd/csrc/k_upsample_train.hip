// Training step of the upsampling network (Sec. 5.2): loss, hand-written
// backward and AdamW with global-norm gradient clipping, on a batch of
// (RGB, code) pairs drawn by index.  Deterministic: fixed summation orders,
// no floating-point atomics.
//
//   1. partials: a workgroup takes two samples at a time, one per half
//                (128 threads, one per hidden unit).  Forward through the
//                three layers, the per-sample loss terms and dL/dz, then
//                backward to the hidden pre-activations, with W2 and W3 in LDS
//                (odd row stride: row-wise and column-wise reads are both
//                conflict-free).  Every thread owns a fixed set of gradient
//                elements and accumulates them over the workgroup's samples
//                in registers; one partial row per workgroup.
//   2. reduce  : a lane per parameter sums the partial rows in a fixed order
//                (float64), divides by N, writes the gradient, and each block
//                writes its sum of squares; block 0 also sums the loss.
//   3. adamw   : every block forms the global gradient norm from the block
//                sums (same order everywhere), the clipping factor
//                min(1, max_norm / (norm + 1e-6)), then per parameter the
//                decoupled weight decay and the Adam update.

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kH = 128;            // hidden width
constexpr int kThreads = 256;
constexpr int kRS = kH + 1;        // LDS row stride of W2 and W3
constexpr int kMaxRows = 128;      // partial rows (workgroups of kernel 1)
constexpr int kW3PerThread = kMaxK / 2;

// packed parameter offsets (floats): W1 (128 x 3), b1, W2 (128 x 128), b2, W3 (k x 128), b3
constexpr int64_t kOffB1 = 3 * kH;
constexpr int64_t kOffW2 = kOffB1 + kH;
constexpr int64_t kOffB2 = kOffW2 + kH * kH;
constexpr int64_t kOffW3 = kOffB2 + kH;
__host__ __device__ inline int64_t off_b3(int k) { return kOffW3 + int64_t(k) * kH; }
__host__ __device__ inline int64_t param_count(int k) { return off_b3(k) + k; }

struct TrainArgs {
    int k;
    const float* params;
    const float* rgb;
    int64_t ld_rgb;
    const float* zgt;
    int64_t ld_z;
    int64_t rows;
    const uint32_t* idx;
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

__global__ __launch_bounds__(kThreads) void ustrain_partials_kernel(TrainArgs a) {
    extern __shared__ __align__(16) float sm[];
    const int k = a.k;
    float* sW2 = sm;                    // 128 x kRS
    float* sW3 = sW2 + kH * kRS;        // k x kRS
    float* sW1 = sW3 + k * kRS;         // 128 x 4 (w_r, w_g, w_b, b1)
    float* sB2 = sW1 + 4 * kH;
    float* sB3 = sB2 + kH;              // k
    float* sM = sB3 + kMaxK;            // 3 x k
    float* sS = sM + 3 * kMaxK;         // per half: p1, h1, p2, h2, dp2, dp1 (128 each), z, d, dz (48 each), misc 8
    constexpr int kHalf = 6 * kH + 3 * kMaxK + 8;

    const int tid = threadIdx.x;
    const float* P = a.params;
    for (int e = tid; e < kH * kH; e += kThreads) sW2[(e / kH) * kRS + e % kH] = P[kOffW2 + e];
    for (int e = tid; e < k * kH; e += kThreads) sW3[(e / kH) * kRS + e % kH] = P[kOffW3 + e];
    for (int j = tid; j < kH; j += kThreads) {
        sW1[4 * j + 0] = P[3 * j];
        sW1[4 * j + 1] = P[3 * j + 1];
        sW1[4 * j + 2] = P[3 * j + 2];
        sW1[4 * j + 3] = P[kOffB1 + j];
        sB2[j] = P[kOffB2 + j];
    }
    for (int c = tid; c < k; c += kThreads) sB3[c] = P[off_b3(k) + c];
    for (int e = tid; e < 3 * k; e += kThreads) sM[e] = a.M[e];

    const int half = tid / kH, j = tid % kH;
    float* S = sS + half * kHalf;
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
    float* SA = sS;            // the two halves' areas for the accumulation phase
    float* SB = sS + kHalf;

    // gradient elements owned by this thread
    float aW2[64];
#pragma unroll
    for (int q = 0; q < 64; ++q) aW2[q] = 0.f;
    float aW3[kW3PerThread];
#pragma unroll
    for (int r = 0; r < kW3PerThread; ++r) aW3[r] = 0.f;
    float aB = 0.f, aW1[3] = {0.f, 0.f, 0.f}, aB3 = 0.f;
    double loss = 0.0;
    __syncthreads();

    const int64_t pairs = (a.N + 1) / 2;
    for (int64_t pr = blockIdx.x; pr < pairs; pr += gridDim.x) {
        const int64_t s = 2 * pr + half;
        const bool valid = s < a.N;
        int64_t row = 0;
        if (valid) row = a.idx ? min<int64_t>(a.idx[s], a.rows - 1) : s;
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
            for (int i = 0; i < kH; ++i) v = fmaf(sW2[j * kRS + i], h1[i], v);
            p2[j] = v;
            h2[j] = v * logistic(v);
        }
        __syncthreads();
        if (j < k) {
            float v = sB3[j];
            for (int i = 0; i < kH; ++i) v = fmaf(sW3[j * kRS + i], h2[i], v);
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
        // accumulate both samples into the owned gradient elements
        {
            const int jj = tid % kH, hi = tid / kH;
            const float h1a = SA[kH + jj], h1b = SB[kH + jj];
#pragma unroll
            for (int q = 0; q < 64; ++q) {
                const int i = 2 * q + hi;
                aW2[q] = fmaf(SA[4 * kH + i], h1a, fmaf(SB[4 * kH + i], h1b, aW2[q]));
            }
            const float h2a = SA[3 * kH + jj], h2b = SB[3 * kH + jj];
            const float* dza = SA + 6 * kH + 2 * kMaxK;
            const float* dzb = SB + 6 * kH + 2 * kMaxK;
#pragma unroll
            for (int r = 0; r < kW3PerThread; ++r) {
                const int c = 2 * r + hi;
                if (c < k) aW3[r] = fmaf(dza[c], h2a, fmaf(dzb[c], h2b, aW3[r]));
            }
            if (hi == 0) {
                aB += SA[4 * kH + jj] + SB[4 * kH + jj];  // b2
            } else {
                const float da = SA[5 * kH + jj], db = SB[5 * kH + jj];
                const float* ma = SA + 6 * kH + 3 * kMaxK;
                const float* mb = SB + 6 * kH + 3 * kMaxK;
#pragma unroll
                for (int x = 0; x < 3; ++x) aW1[x] = fmaf(da, ma[x], fmaf(db, mb[x], aW1[x]));
                aB += da + db;  // b1
            }
            if (tid < k) aB3 += dza[tid] + dzb[tid];
        }
        __syncthreads();
    }
    // partial row
    float* prow = a.part + int64_t(blockIdx.x) * param_count(k);
    {
        const int jj = tid % kH, hi = tid / kH;
#pragma unroll
        for (int q = 0; q < 64; ++q) prow[kOffW2 + (2 * q + hi) * kH + jj] = aW2[q];
#pragma unroll
        for (int r = 0; r < kW3PerThread; ++r) {
            const int c = 2 * r + hi;
            if (c < k) prow[kOffW3 + c * kH + jj] = aW3[r];
        }
        if (hi == 0) {
            prow[kOffB2 + jj] = aB;
        } else {
#pragma unroll
            for (int x = 0; x < 3; ++x) prow[3 * jj + x] = aW1[x];
            prow[kOffB1 + jj] = aB;
        }
        if (tid < k) prow[off_b3(k) + tid] = aB3;
    }
    // workgroup loss: the two per-sample threads (tid 0 and 128), fixed order
    __shared__ double s_loss[2];
    if (tid % kH == 0) s_loss[tid / kH] = loss;
    __syncthreads();
    if (tid == 0) a.loss_part[blockIdx.x] = s_loss[0] + s_loss[1];
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

__global__ __launch_bounds__(kThreads) void ustrain_reduce_kernel(ReduceArgs a) {
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    double g = 0.0;
    if (e < a.P) {
        // eight interleaved partial sums keep eight row loads in flight
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int r = 0;
        for (; r + 8 <= a.rows; r += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += double(a.part[int64_t(r + u) * a.P + e]);
        }
        for (; r < a.rows; ++r) acc[0] += double(a.part[int64_t(r) * a.P + e]);
        const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        g = s / double(a.N);
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
        if (blockIdx.x == 0) {
            double l = 0.0;
            for (int r = 0; r < a.rows; ++r) l += a.loss_part[r];
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
};

__global__ __launch_bounds__(kThreads) void ustrain_adamw_kernel(AdamWArgs a) {
    __shared__ double s_scale;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < a.nsq; ++b) t += a.sq_part[b];
        const double norm = sqrt(t);
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
    const double bc1 = 1.0 - pow(a.beta1, t);
    const double bc2 = 1.0 - pow(a.beta2, t);
    a.m[e] = float(mm);
    a.v[e] = float(vv);
    a.params[e] = float(w - (a.lr / bc1) * mm / (sqrt(vv) / sqrt(bc2) + a.eps));
}

int64_t grid_rows(int64_t N) { return std::min<int64_t>((N + 1) / 2, kMaxRows); }

size_t lds_bytes(int k) {
    return sizeof(float) * (size_t(kH) * kRS + size_t(k) * kRS + 4 * kH + kH + kMaxK + 3 * kMaxK +
                            2 * (6 * kH + 3 * kMaxK + 8));
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
    a.N = u.N;
    a.M = u.M;
    a.wx = float(u.white[0]);
    a.wy = float(u.white[1]);
    a.wz = float(u.white[2]);
    a.w_max = float(u.w_max);
    a.w_col = float(u.w_col);
    a.part = ws.part;
    a.loss_part = ws.loss_part;
    hipLaunchKernelGGL(ustrain_partials_kernel, dim3(uint32_t(rows)), dim3(kThreads), lds_bytes(k), st, a);
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
    w.eps = u.opt->eps;
    w.wd = u.opt->weight_decay;
    w.max_norm = u.opt->max_grad_norm;
    hipLaunchKernelGGL(ustrain_adamw_kernel, dim3(nsq), dim3(kThreads), 0, st, w);
    return launch_status("hc_upsample_train_step");
}

}  // namespace hc
