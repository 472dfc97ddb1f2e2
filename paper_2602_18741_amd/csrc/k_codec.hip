// Codec fitting: loss, hand-written gradient and Adam for the non-negative
// linear codec E = softplus(Wt_E), D = softplus(Wt_D).
//
// Up to three kernels per step, all deterministic (fixed summation orders,
// no floating-point atomics):
//   1. weights : E, D = softplus_beta(Wt) into the workspace; bumps the Adam
//                step counter.  Only when E and D do not fit the partials
//                kernel's LDS; otherwise that kernel stages softplus(Wt)
//                itself and its block 0 bumps the counter.
//   2. partials: each workgroup takes tiles of TP pairs; `lpp` lanes per pair
//                compute u = E a, v = E b, h = u*v, the residuals
//                r_a = D u - a, r_b = D v - b, r_h = D h - a*b, and the
//                back-propagated code gradients, staged in LDS; then every
//                thread contracts over the tile's pairs for its gradient
//                elements (in the parameters' precision over the tile's at
//                most 64 pairs, in float64 across tiles) and writes one
//                partial row per workgroup.  One kernel per objective: the two-term squared
//                error, or the four-term loss of Eq. 8 (which also needs the
//                per-pair norms and dot product of the cosine factor, reduced
//                across the pair's lanes by shuffles, and the code of the
//                spectral product for L_code).
//   3. finish  : one wavefront per gradient element sums the partial rows
//                (fixed order, float64), scales by 2/N (two-term) or 1/N
//                (Eq. 8, whose per-pair terms carry their own factors),
//                applies the softplus slope logistic(beta Wt) and optionally
//                the Adam update.

#include "hc_internal.hpp"

namespace hc {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxRows = 1024;          // partial rows (workgroups of kernel 2)
constexpr size_t kTileLdsBytes = 49152;

__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dlog1p(float x) { return log1pf(x); }
__device__ __forceinline__ double dlog1p(double x) { return log1p(x); }

template <typename F>
__device__ __forceinline__ F softplus(F x, F beta) {
    const F ax = x < F(0) ? -x : x;
    return (x > F(0) ? x : F(0)) + dlog1p(dexp(-beta * ax)) / beta;
}

// logistic(beta x), the slope of softplus_beta at x
__device__ __forceinline__ double slope(double x, double beta) {
    const double e = exp(-beta * (x < 0 ? -x : x));
    return x >= 0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

// ------------------------------------------------------------------ kernel 1

template <typename F>
__global__ __launch_bounds__(kThreads) void codec_weights_kernel(const F* we, const F* wd, int kn,
                                                                 F beta, F* E, F* D,
                                                                 int64_t* step, int64_t* ws_step) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e < kn) {
        E[e] = softplus(we[e], beta);
        D[e] = softplus(wd[e], beta);
    }
    if (step && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t t = *step + 1;
        *ws_step = t;
        *step = t;
    }
}

template <typename F>
__global__ __launch_bounds__(kThreads) void codec_weights_f32_kernel(const F* we, const F* wd, int kn,
                                                                     F beta, float* E, float* D) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e < kn) {
        E[e] = float(softplus(we[e], beta));
        D[e] = float(softplus(wd[e], beta));
    }
}

// ------------------------------------------------------------------ kernel 2

template <typename F>
struct PartialArgs {
    int k, n, npad, tp, lpp;
    F lam;
    const F* E;  // k x n
    const F* D;  // n x k
    const F* A;
    const F* B;
    int64_t ld_a, ld_b, rows_a, rows_b;
    const uint32_t* idx_a;
    const uint32_t* idx_b;
    int64_t N, n_tiles;
    double* part;  // gridDim.x rows of 2kn + 1
    int ed_in_lds;
    // with E and D staged in LDS the kernel makes them itself from the raw
    // parameters (softplus), and block 0 bumps the Adam step counter: the
    // weights kernel is then not launched
    const F* we;
    const F* wd;
    F beta;
    int64_t* step;
    int64_t* ws_step;
    // Eq. 8 objective
    const F* T;  // 3 x n
    double w_e2e, w_rec, w_code, w_col, eps;
};

// E = softplus(Wt_E) and D = softplus(Wt_D) into LDS (the values the weights
// kernel would write), and the step counter bump.
template <typename F>
__device__ __forceinline__ void stage_weights(const PartialArgs<F>& a, F* sm, int kn) {
    for (int i = threadIdx.x; i < kn; i += kThreads) {
        sm[i] = softplus(a.we[i], a.beta);
        sm[kn + i] = softplus(a.wd[i], a.beta);
    }
    if (a.step && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t t = *a.step + 1;
        *a.ws_step = t;
        *a.step = t;
    }
}

template <typename F>
__global__ __launch_bounds__(kThreads) void codec_partials_kernel(PartialArgs<F> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    F* sm = reinterpret_cast<F*>(smem_raw);
    const int k = a.k, n = a.n, np = a.npad, tp = a.tp, lpp = a.lpp;
    const int kn = k * n;
    const int tid = threadIdx.x;
    const F* Ep = a.E;
    const F* Dp = a.D;
    F* base = sm;
    if (a.ed_in_lds) {
        stage_weights(a, sm, kn);
        Ep = sm;
        Dp = sm + kn;
        base = sm + 2 * kn;
    }
    F* AA = base;
    F* BB = AA + tp * np;
    F* RA = BB + tp * np;
    F* RB = RA + tp * np;
    F* RH = RB + tp * np;
    F* U = RH + tp * np;
    F* V = U + tp * k;
    F* H = V + tp * k;
    F* GU = H + tp * k;
    F* GV = GU + tp * k;

    const int pair = tid / lpp;
    const int part = tid % lpp;
    double loss_acc = 0.0;
    double* prow = a.part + int64_t(blockIdx.x) * (2 * kn + 1);
    bool first_tile = true;

    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const int64_t gi = tile * tp + pair;
        const bool valid = pair < tp && gi < a.N;
        __syncthreads();  // the previous tile's contraction has finished with LDS
        if (pair < tp) {
            int64_t ra = 0, rb = 0;
            if (valid) {
                ra = a.idx_a ? min<int64_t>(a.idx_a[gi], a.rows_a - 1) : gi;
                rb = a.idx_b ? min<int64_t>(a.idx_b[gi], a.rows_b - 1) : gi;
            }
            for (int i = part; i < n; i += lpp) {
                AA[pair * np + i] = valid ? a.A[ra * a.ld_a + i] : F(0);
                BB[pair * np + i] = valid ? a.B[rb * a.ld_b + i] : F(0);
            }
        }
        __syncthreads();
        // codes u = E a, v = E b and their product h (Eq. 4, Eq. 6)
        if (pair < tp) {
            for (int j = part; j < k; j += lpp) {
                F su = 0, sv = 0;
                for (int i = 0; i < n; ++i) {
                    const F e = Ep[j * n + i];
                    su += e * AA[pair * np + i];
                    sv += e * BB[pair * np + i];
                }
                U[pair * k + j] = su;
                V[pair * k + j] = sv;
                H[pair * k + j] = su * sv;
            }
        }
        __syncthreads();
        // residuals of the two reconstructions and of the decoded product
        if (pair < tp) {
            for (int i = part; i < n; i += lpp) {
                F du = 0, dv = 0, dh = 0;
                for (int j = 0; j < k; ++j) {
                    const F d = Dp[i * k + j];
                    du += d * U[pair * k + j];
                    dv += d * V[pair * k + j];
                    dh += d * H[pair * k + j];
                }
                const F ai = AA[pair * np + i], bi = BB[pair * np + i];
                const F ra = du - ai, rb = dv - bi, rh = dh - ai * bi;
                if (valid)
                    loss_acc += double(ra) * double(ra) + double(rb) * double(rb) +
                                double(a.lam) * double(rh) * double(rh);
                RA[pair * np + i] = valid ? ra : F(0);
                RB[pair * np + i] = valid ? rb : F(0);
                RH[pair * np + i] = valid ? a.lam * rh : F(0);
            }
        }
        __syncthreads();
        // code-space gradients: D^T r_a + g_h * v and D^T r_b + g_h * u with g_h = lam D^T r_h
        if (pair < tp) {
            for (int j = part; j < k; j += lpp) {
                F gu = 0, gv = 0, gh = 0;
                for (int i = 0; i < n; ++i) {
                    const F d = Dp[i * k + j];
                    gu += d * RA[pair * np + i];
                    gv += d * RB[pair * np + i];
                    gh += d * RH[pair * np + i];
                }
                GU[pair * k + j] = gu + gh * V[pair * k + j];
                GV[pair * k + j] = gv + gh * U[pair * k + j];
            }
        }
        __syncthreads();
        // contraction over the tile's pairs; elements [0, kn) are dL/dE
        // (k x n), [kn, 2kn) are dL/dD (n x k), both without the 2/N factor
        for (int e = tid; e < 2 * kn; e += kThreads) {
            F s = 0;
            if (e < kn) {
                const int j = e / n, i = e % n;
                for (int p = 0; p < tp; ++p)
                    s += GU[p * k + j] * AA[p * np + i] + GV[p * k + j] * BB[p * np + i];
            } else {
                const int e2 = e - kn;
                const int i = e2 / k, j = e2 % k;
                for (int p = 0; p < tp; ++p)
                    s += RA[p * np + i] * U[p * k + j] + RB[p * np + i] * V[p * k + j] +
                         RH[p * np + i] * H[p * k + j];
            }
            prow[e] = first_tile ? double(s) : prow[e] + double(s);
        }
        first_tile = false;
    }
    // workgroup sum of the loss terms, fixed order
    __shared__ double s_loss[kThreads / kWave];
    for (int m = kWave / 2; m >= 1; m >>= 1) loss_acc += __shfl_xor(loss_acc, m, kWave);
    if ((tid & (kWave - 1)) == 0) s_loss[tid / kWave] = loss_acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) t += s_loss[w];
        prow[2 * kn] = t;
    }
}


// Four-term objective of Eq. 8.  Per pair (a, b), t = a*b:
//   S = D h, r_h = S - t, M = |r_h|^2 / n, c = cos(S, t) with clamped norms,
//   r_c = T r_h, d = h - E t;
//   loss = w_e2e M (2 - c) + w_rec (|r_a|^2 + |r_b|^2)/n + w_code |d|^2/k + w_col |r_c|^2/3
// Backward (per pair, summed here, / N in the finish kernel):
//   g_S = w_e2e ((2 - c)(2/n) r_h - M dc/dS) + w_col (2/3) T^T r_c,
//   dc/dS = t/(|S| m_t) - c S/|S|^2 if |S| > eps else t/(eps m_t), m_t = max(|t|, eps)
//   g_h = D^T g_S + w_code (2/k) d,
//   g_u = w_rec (2/n) D^T r_a + g_h*v, g_v = w_rec (2/n) D^T r_b + g_h*u
//   dE += g_u a^T + g_v b^T - w_code (2/k) d t^T
//   dD += w_rec (2/n)(r_a u^T + r_b v^T) + g_S h^T
template <typename F>
__global__ __launch_bounds__(kThreads) void codec_partials_eq8_kernel(PartialArgs<F> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    F* sm = reinterpret_cast<F*>(smem_raw);
    const int k = a.k, n = a.n, np = a.npad, tp = a.tp, lpp = a.lpp;
    const int kn = k * n;
    const int tid = threadIdx.x;
    const F* Ep = a.E;
    const F* Dp = a.D;
    F* base = sm;
    if (a.ed_in_lds) {
        stage_weights(a, sm, kn);
        Ep = sm;
        Dp = sm + kn;
        base = sm + 2 * kn;
    }
    F* AA = base;          // a
    F* BB = AA + tp * np;  // b
    F* TT = BB + tp * np;  // t = a*b
    F* RA = TT + tp * np;  // r_a, then w_rec (2/n) r_a
    F* RB = RA + tp * np;
    F* SG = RB + tp * np;  // S, then g_S
    F* U = SG + tp * np;
    F* V = U + tp * k;
    F* H = V + tp * k;
    F* DC = H + tp * k;    // d = h - E t, then w_code (2/k) d
    F* GU = DC + tp * k;
    F* GV = GU + tp * k;

    const int pair = tid / lpp;
    const int part = tid % lpp;
    const double inv_n = 1.0 / n;
    double loss_acc = 0.0;
    double* prow = a.part + int64_t(blockIdx.x) * (2 * kn + 1);
    bool first_tile = true;

    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const int64_t gi = tile * tp + pair;
        const bool valid = gi < a.N;
        __syncthreads();  // the previous tile's contraction has finished with LDS
        {
            int64_t ra = 0, rb = 0;
            if (valid) {
                ra = a.idx_a ? min<int64_t>(a.idx_a[gi], a.rows_a - 1) : gi;
                rb = a.idx_b ? min<int64_t>(a.idx_b[gi], a.rows_b - 1) : gi;
            }
            for (int i = part; i < n; i += lpp) {
                const F ai = valid ? a.A[ra * a.ld_a + i] : F(0);
                const F bi = valid ? a.B[rb * a.ld_b + i] : F(0);
                AA[pair * np + i] = ai;
                BB[pair * np + i] = bi;
                TT[pair * np + i] = ai * bi;
            }
        }
        __syncthreads();
        // codes u = E a, v = E b, their product h (Eq. 4, Eq. 6), and d = h - E t
        for (int j = part; j < k; j += lpp) {
            F su = 0, sv = 0, st = 0;
            for (int i = 0; i < n; ++i) {
                const F e = Ep[j * n + i];
                su += e * AA[pair * np + i];
                sv += e * BB[pair * np + i];
                st += e * TT[pair * np + i];
            }
            U[pair * k + j] = su;
            V[pair * k + j] = sv;
            H[pair * k + j] = su * sv;
            DC[pair * k + j] = su * sv - st;
        }
        __syncthreads();
        // reconstructions; per-lane partial sums of the pair's norms
        double s_rr = 0, s_rh = 0, s_st = 0, s_ss = 0, s_tt = 0, s_c0 = 0, s_c1 = 0, s_c2 = 0, s_dd = 0;
        for (int i = part; i < n; i += lpp) {
            F du = 0, dv = 0, dh = 0;
            for (int j = 0; j < k; ++j) {
                const F d = Dp[i * k + j];
                du += d * U[pair * k + j];
                dv += d * V[pair * k + j];
                dh += d * H[pair * k + j];
            }
            const F ra = du - AA[pair * np + i], rb = dv - BB[pair * np + i];
            const F ti = TT[pair * np + i];
            const F rh = dh - ti;
            RA[pair * np + i] = ra;
            RB[pair * np + i] = rb;
            SG[pair * np + i] = dh;
            s_rr += double(ra) * double(ra) + double(rb) * double(rb);
            s_rh += double(rh) * double(rh);
            s_st += double(dh) * double(ti);
            s_ss += double(dh) * double(dh);
            s_tt += double(ti) * double(ti);
            s_c0 += double(a.T[i]) * double(rh);
            s_c1 += double(a.T[n + i]) * double(rh);
            s_c2 += double(a.T[2 * n + i]) * double(rh);
        }
        for (int j = part; j < k; j += lpp) s_dd += double(DC[pair * k + j]) * double(DC[pair * k + j]);
        // reduce over the pair's lpp consecutive lanes (lpp divides the wavefront)
        for (int m = 1; m < lpp; m <<= 1) {
            s_rr += __shfl_xor(s_rr, m, kWave);
            s_rh += __shfl_xor(s_rh, m, kWave);
            s_st += __shfl_xor(s_st, m, kWave);
            s_ss += __shfl_xor(s_ss, m, kWave);
            s_tt += __shfl_xor(s_tt, m, kWave);
            s_c0 += __shfl_xor(s_c0, m, kWave);
            s_c1 += __shfl_xor(s_c1, m, kWave);
            s_c2 += __shfl_xor(s_c2, m, kWave);
            s_dd += __shfl_xor(s_dd, m, kWave);
        }
        const double M = s_rh * inv_n;
        const double sn = sqrt(s_ss);
        const double ns = sn > a.eps ? sn : a.eps;
        const double tn = sqrt(s_tt);
        const double nt = tn > a.eps ? tn : a.eps;
        const double c = s_st / (ns * nt);
        if (valid && part == 0)
            loss_acc += a.w_e2e * M * (2.0 - c) + a.w_rec * s_rr * inv_n + a.w_code * s_dd / k +
                        a.w_col * (s_c0 * s_c0 + s_c1 * s_c1 + s_c2 * s_c2) / 3.0;
        // g_S = al r_h - bt t + bs S + T^T gc; r_a, r_b scaled by w_rec (2/n)
        const F al = F(a.w_e2e * (2.0 - c) * 2.0 * inv_n);
        const F bt = F(a.w_e2e * M / (ns * nt));
        const F bs = F(sn > a.eps ? a.w_e2e * M * c / s_ss : 0.0);
        const F g0 = F(a.w_col * (2.0 / 3.0) * s_c0), g1 = F(a.w_col * (2.0 / 3.0) * s_c1),
                g2 = F(a.w_col * (2.0 / 3.0) * s_c2);
        const F wr = F(a.w_rec * 2.0 * inv_n);
        for (int i = part; i < n; i += lpp) {
            const F S = SG[pair * np + i], ti = TT[pair * np + i];
            const F gs = al * (S - ti) - bt * ti + bs * S + g0 * a.T[i] + g1 * a.T[n + i] +
                         g2 * a.T[2 * n + i];
            SG[pair * np + i] = valid ? gs : F(0);
            RA[pair * np + i] = valid ? wr * RA[pair * np + i] : F(0);
            RB[pair * np + i] = valid ? wr * RB[pair * np + i] : F(0);
        }
        __syncthreads();
        // code-space gradients
        const F wk = F(a.w_code * 2.0 / k);
        for (int j = part; j < k; j += lpp) {
            F gu = 0, gv = 0, gs = 0;
            for (int i = 0; i < n; ++i) {
                const F d = Dp[i * k + j];
                gu += d * RA[pair * np + i];
                gv += d * RB[pair * np + i];
                gs += d * SG[pair * np + i];
            }
            const F dc = valid ? wk * DC[pair * k + j] : F(0);
            const F gh = gs + dc;
            DC[pair * k + j] = dc;
            GU[pair * k + j] = gu + gh * V[pair * k + j];
            GV[pair * k + j] = gv + gh * U[pair * k + j];
        }
        __syncthreads();
        // contraction over the tile's pairs; [0, kn) is dL/dE, [kn, 2kn) dL/dD
        for (int e = tid; e < 2 * kn; e += kThreads) {
            F s = 0;
            if (e < kn) {
                const int j = e / n, i = e % n;
                for (int p = 0; p < tp; ++p)
                    s += GU[p * k + j] * AA[p * np + i] + GV[p * k + j] * BB[p * np + i] -
                         DC[p * k + j] * TT[p * np + i];
            } else {
                const int e2 = e - kn;
                const int i = e2 / k, j = e2 % k;
                for (int p = 0; p < tp; ++p)
                    s += RA[p * np + i] * U[p * k + j] + RB[p * np + i] * V[p * k + j] +
                         SG[p * np + i] * H[p * k + j];
            }
            prow[e] = first_tile ? double(s) : prow[e] + double(s);
        }
        first_tile = false;
    }
    __shared__ double s_loss[kThreads / kWave];
    for (int m = kWave / 2; m >= 1; m >>= 1) loss_acc += __shfl_xor(loss_acc, m, kWave);
    if ((tid & (kWave - 1)) == 0) s_loss[tid / kWave] = loss_acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) t += s_loss[w];
        prow[2 * kn] = t;
    }
}

// ------------------------------------------------------------------ kernel 3

template <typename F>
struct FinishArgs {
    int k, n;
    double beta, inv_n, gscale;
    const double* part;
    int rows;
    F* we;
    F* wd;
    F* loss;
    F* grad_e;
    F* grad_d;
    // Adam
    F* m_e;
    F* v_e;
    F* m_d;
    F* v_d;
    const int64_t* ws_step;
    double lr, beta1, beta2, eps;
    int adam;
};

template <typename F>
__global__ __launch_bounds__(kThreads) void codec_finish_kernel(FinishArgs<F> a) {
    const int kn = a.k * a.n;
    const int lane = threadIdx.x & (kWave - 1);
    const int e = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
    if (e > 2 * kn) return;
    const int64_t stride = 2 * kn + 1;
    // eight interleaved partial sums per lane keep eight row loads in flight
    // (the rows of one element are a column: every load is its own line)
    constexpr int kIlp = 8;
    double acc[kIlp];
#pragma unroll
    for (int u = 0; u < kIlp; ++u) acc[u] = 0.0;
    int r = lane;
    for (; r + (kIlp - 1) * kWave < a.rows; r += kIlp * kWave) {
        double v[kIlp];
#pragma unroll
        for (int u = 0; u < kIlp; ++u) v[u] = a.part[int64_t(r + u * kWave) * stride + e];
#pragma unroll
        for (int u = 0; u < kIlp; ++u) acc[u] += v[u];
    }
    for (; r < a.rows; r += kWave) acc[0] += a.part[int64_t(r) * stride + e];
    double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    for (int m = kWave / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, kWave);
    if (lane != 0) return;
    if (e == 2 * kn) {
        *a.loss = F(s * a.inv_n);
        return;
    }
    const bool isE = e < kn;
    const int idx = isE ? e : e - kn;
    F* w = isE ? a.we : a.wd;
    const double wt = double(w[idx]);
    const double g = s * a.gscale * slope(wt, a.beta);
    F* gout = isE ? a.grad_e : a.grad_d;
    if (gout) gout[idx] = F(g);
    if (a.adam) {
        F* m = isE ? a.m_e : a.m_d;
        F* v = isE ? a.v_e : a.v_d;
        const double t = double(*a.ws_step);
        const double mm = a.beta1 * double(m[idx]) + (1.0 - a.beta1) * g;
        const double vv = a.beta2 * double(v[idx]) + (1.0 - a.beta2) * g * g;
        const double bc1 = 1.0 - pow(a.beta1, t);
        const double bc2 = 1.0 - pow(a.beta2, t);
        const double denom = sqrt(vv) / sqrt(bc2) + a.eps;
        m[idx] = F(mm);
        v[idx] = F(vv);
        w[idx] = F(wt - (a.lr / bc1) * mm / denom);
    }
}

// ------------------------------------------------------------------ host side

struct Plan {
    int tp, lpp, npad, ed_in_lds;
    int64_t n_tiles, grid;
    size_t lds;
};

Plan plan(int k, int n, int64_t N, size_t esz, int objective) {
    Plan p;
    p.npad = n | 1;  // odd row stride spreads the pairs of a wave over LDS banks
    const size_t ed = size_t(2) * k * n * esz;
    p.ed_in_lds = ed <= 16384;
    const size_t rows_n = objective == HC_CODEC_EQ8 ? 6 : 5, rows_k = rows_n;
    const size_t per_pair = (rows_n * p.npad + rows_k * k) * esz;
    const size_t budget = kTileLdsBytes - (p.ed_in_lds ? ed : 0);
    int tp = 64;
    while (tp > 4 && size_t(tp) * per_pair > budget) tp >>= 1;
    p.tp = tp;
    p.lpp = kThreads / tp;
    p.lds = size_t(tp) * per_pair + (p.ed_in_lds ? ed : 0);
    p.n_tiles = ceil_div(N, tp);
    p.grid = std::min<int64_t>(p.n_tiles, kMaxRows);
    return p;
}

size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

struct Workspace {
    void* E;
    void* D;
    double* part;
    int64_t* step;
};

Workspace carve(void* ws, int k, int n, int64_t rows, size_t esz) {
    char* p = static_cast<char*>(ws);
    Workspace w;
    const size_t kn = size_t(k) * n;
    w.E = p;
    p += align8(kn * esz);
    w.D = p;
    p += align8(kn * esz);
    w.part = reinterpret_cast<double*>(p);
    p += size_t(rows) * (2 * kn + 1) * sizeof(double);
    w.step = reinterpret_cast<int64_t*>(p);
    return w;
}

template <typename F>
hc_status run(const hc_codec_args& a) {
    const int k = a.k, n = a.n, kn = k * n;
    hipStream_t st = reinterpret_cast<hipStream_t>(a.stream);
    const bool eq8 = a.objective == HC_CODEC_EQ8;
    const Plan pl = plan(k, n, a.N, sizeof(F), a.objective);
    Workspace ws = carve(a.workspace, k, n, pl.grid, sizeof(F));
    int64_t* adam_step = a.adam ? a.adam->step : nullptr;
    hc_status s = HC_OK;
    if (!pl.ed_in_lds) {
        // the partials kernel reads E and D from the workspace
        const int g0 = int(ceil_div(kn, kThreads));
        hipLaunchKernelGGL(codec_weights_kernel<F>, dim3(g0), dim3(kThreads), 0, st,
                           static_cast<const F*>(a.Wt_E), static_cast<const F*>(a.Wt_D), kn,
                           F(a.beta), static_cast<F*>(ws.E), static_cast<F*>(ws.D), adam_step, ws.step);
        s = launch_status("hc_codec_step");
        if (s != HC_OK) return s;
    }

    PartialArgs<F> p;
    p.k = k;
    p.n = n;
    p.npad = pl.npad;
    p.tp = pl.tp;
    p.lpp = pl.lpp;
    p.lam = F(a.lambda);
    p.E = static_cast<const F*>(ws.E);
    p.D = static_cast<const F*>(ws.D);
    p.A = static_cast<const F*>(a.A);
    p.B = static_cast<const F*>(a.B);
    p.ld_a = a.ld_a;
    p.ld_b = a.ld_b;
    p.rows_a = a.rows_a;
    p.rows_b = a.rows_b;
    p.idx_a = a.idx_a;
    p.idx_b = a.idx_b;
    p.N = a.N;
    p.n_tiles = pl.n_tiles;
    p.part = ws.part;
    p.ed_in_lds = pl.ed_in_lds;
    p.we = static_cast<const F*>(a.Wt_E);
    p.wd = static_cast<const F*>(a.Wt_D);
    p.beta = F(a.beta);
    p.step = pl.ed_in_lds ? adam_step : nullptr;
    p.ws_step = ws.step;
    p.T = static_cast<const F*>(a.T);
    p.w_e2e = a.w_e2e;
    p.w_rec = a.w_rec;
    p.w_code = a.w_code;
    p.w_col = a.w_col;
    p.eps = a.cos_eps;
    if (eq8)
        hipLaunchKernelGGL(codec_partials_eq8_kernel<F>, dim3(uint32_t(pl.grid)), dim3(kThreads), pl.lds,
                           st, p);
    else
        hipLaunchKernelGGL(codec_partials_kernel<F>, dim3(uint32_t(pl.grid)), dim3(kThreads), pl.lds, st,
                           p);
    s = launch_status("hc_codec_step");
    if (s != HC_OK) return s;

    FinishArgs<F> f;
    f.k = k;
    f.n = n;
    f.beta = a.beta;
    f.inv_n = 1.0 / double(a.N);
    f.gscale = (eq8 ? 1.0 : 2.0) / double(a.N);
    f.part = ws.part;
    f.rows = int(pl.grid);
    f.we = static_cast<F*>(a.Wt_E);
    f.wd = static_cast<F*>(a.Wt_D);
    f.loss = static_cast<F*>(a.loss);
    f.grad_e = static_cast<F*>(a.grad_E);
    f.grad_d = static_cast<F*>(a.grad_D);
    f.adam = a.adam != nullptr;
    if (a.adam) {
        f.m_e = static_cast<F*>(a.adam->m_E);
        f.v_e = static_cast<F*>(a.adam->v_E);
        f.m_d = static_cast<F*>(a.adam->m_D);
        f.v_d = static_cast<F*>(a.adam->v_D);
        f.lr = a.adam->lr;
        f.beta1 = a.adam->beta1;
        f.beta2 = a.adam->beta2;
        f.eps = a.adam->eps;
    } else {
        f.m_e = f.v_e = f.m_d = f.v_d = nullptr;
        f.lr = f.beta1 = f.beta2 = f.eps = 0.0;
    }
    f.ws_step = ws.step;
    const int g2 = int(ceil_div(2 * kn + 1, kThreads / kWave));
    hipLaunchKernelGGL(codec_finish_kernel<F>, dim3(g2), dim3(kThreads), 0, st, f);
    return launch_status("hc_codec_step");
}

}  // namespace

size_t codec_workspace_size(int k, int n, int64_t N) {
    // the float64 plans have the smallest tiles, hence the most partial rows
    const int64_t rows = std::max(plan(k, n, N, sizeof(double), HC_CODEC_L2).grid,
                                  plan(k, n, N, sizeof(double), HC_CODEC_EQ8).grid);
    const size_t kn = size_t(k) * n;
    return 2 * align8(kn * sizeof(double)) + size_t(rows) * (2 * kn + 1) * sizeof(double) +
           sizeof(int64_t);
}

hc_status launch_codec_step(const hc_codec_args& a) {
    return a.dtype == 1 ? run<double>(a) : run<float>(a);
}

hc_status launch_codec_weights(const void* we, const void* wd, int k, int n, int dtype, double beta,
                               float* E, float* D, hipStream_t st) {
    const int kn = k * n;
    const int g = int(ceil_div(kn, kThreads));
    if (dtype == 1)
        hipLaunchKernelGGL(codec_weights_f32_kernel<double>, dim3(g), dim3(kThreads), 0, st,
                           static_cast<const double*>(we), static_cast<const double*>(wd), kn, beta,
                           E, D);
    else
        hipLaunchKernelGGL(codec_weights_f32_kernel<float>, dim3(g), dim3(kThreads), 0, st,
                           static_cast<const float*>(we), static_cast<const float*>(wd), kn,
                           float(beta), E, D);
    return launch_status("hc_codec_weights");
}

}  // namespace hc
