// Codec fitting: loss, hand-written gradient and Adam for the non-negative
// linear codec E = softplus(Wt_E), D = softplus(Wt_D).
//
// Two or three kernels per step, all deterministic (fixed summation orders,
// no floating-point atomics).  The batch rows come from the caller, through
// index arrays, or from the counter-based generator inside the partials
// kernel.
//   1. weights : E, D = softplus_beta(Wt) into the workspace, and the
//                incremented Adam step into the workspace.  Only when E and D
//                do not fit the partials kernel's LDS; otherwise that kernel
//                stages softplus(Wt) itself and its block 0 writes the step.
//   2. partials, float32 with n = 31 and k = 6 or 9: two lanes per pair
//                with the pair in registers and the sums over pairs of outer
//                products on the fp32 matrix cores (kernel 2 below, "a few
//                lanes per pair"); float32 with n = 81 and k = 6 or 9: every
//                product on the matrix cores, 16 pairs per wavefront tile
//                (kernel 2 below, "matrix-core tiles").  Otherwise each workgroup takes
//                tiles of TP pairs; `lpp` lanes per pair compute u = E a,
//                v = E b, h = u*v, the residuals r_a = D u - a, r_b = D v - b,
//                r_h = D h - a*b, and the back-propagated code gradients,
//                staged in LDS; then every thread contracts over the tile's
//                pairs for its gradient elements (in the parameters' precision
//                over the tile's at most 64 pairs, in float64 across tiles).
//                Either way one partial row per workgroup.  One kernel per
//                objective: the two-term squared error, or the four-term loss
//                of Eq. 8 (which also needs the per-pair norms and dot product
//                of the cosine factor, reduced across the pair's lanes, and
//                the code of the spectral product for L_code).
//   3. finish  : a workgroup per 64 gradient elements sums the partial rows
//                (fixed order, float64), scales by 2/N (two-term) or 1/N
//                (Eq. 8, whose per-pair terms carry their own factors),
//                applies the softplus slope logistic(beta Wt) and optionally
//                the Adam update, and stores the incremented step counter
//                (after every read of it by the step's pair draw).

#include <cmath>
#include <mutex>
#include <type_traits>

#include "counter_rng.hpp"
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
    if (step && blockIdx.x == 0 && threadIdx.x == 0) *ws_step = *step + 1;
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
    // rows drawn on the device: counter base draw_ctr0 (+ *draw_scale * N)
    int draw;
    uint64_t key_a, key_b, draw_ctr0;
    const int64_t* draw_scale;
    int64_t N, n_tiles;
    double* part;  // gridDim.x rows of 2kn + 1
    int ed_in_lds;
    // with E and D staged in LDS the kernel makes them itself from the raw
    // parameters (softplus), and block 0 writes the incremented Adam step to
    // the workspace: the weights kernel is then not launched
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
// kernel would write), and the incremented step into the workspace (the
// finish kernel stores it to the counter, after every read of the counter
// by this step's pair draw).
template <typename F>
__device__ __forceinline__ void stage_weights(const PartialArgs<F>& a, F* sm, int kn) {
    for (int i = threadIdx.x; i < kn; i += kThreads) {
        sm[i] = softplus(a.we[i], a.beta);
        sm[kn + i] = softplus(a.wd[i], a.beta);
    }
    if (a.step && blockIdx.x == 0 && threadIdx.x == 0) *a.ws_step = *a.step + 1;
}

// Counter base of the pair draw for this call.
template <typename F>
__device__ __forceinline__ uint64_t draw_base(const PartialArgs<F>& a) {
    return a.draw_ctr0 + (a.draw_scale ? uint64_t(*a.draw_scale) * uint64_t(a.N) : 0ull);
}

// Batch rows of pair gi: drawn (the indices hc_gen_indices would write),
// gathered by index (clamped) or the identity.
template <typename F>
__device__ __forceinline__ void batch_rows(const PartialArgs<F>& a, uint64_t base, int64_t gi, int64_t& ra,
                                           int64_t& rb) {
    if (a.draw) {
        ra = range32(rand64(a.key_a, base + uint64_t(gi)), uint64_t(a.rows_a));
        rb = range32(rand64(a.key_b, base + uint64_t(gi)), uint64_t(a.rows_b));
    } else {
        ra = a.idx_a ? min<int64_t>(a.idx_a[gi], a.rows_a - 1) : gi;
        rb = a.idx_b ? min<int64_t>(a.idx_b[gi], a.rows_b - 1) : gi;
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
    const uint64_t ctr_base = a.draw ? draw_base(a) : 0ull;
    double loss_acc = 0.0;
    double* prow = a.part + int64_t(blockIdx.x) * (2 * kn + 1);
    bool first_tile = true;

    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const int64_t gi = tile * tp + pair;
        const bool valid = pair < tp && gi < a.N;
        __syncthreads();  // the previous tile's contraction has finished with LDS
        if (pair < tp) {
            int64_t ra = 0, rb = 0;
            if (valid) batch_rows(a, ctr_base, gi, ra, rb);
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
    const uint64_t ctr_base = a.draw ? draw_base(a) : 0ull;
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
            if (valid) batch_rows(a, ctr_base, gi, ra, rb);
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

// ------------------------------------------------------------------ kernel 2, a few lanes per pair
//
// float32 with n = 31 (400-700 nm at 10 nm) and k = 6 or 9.  LPP = 2
// consecutive lanes of a wavefront own one pair: lane q of the group holds samples
// [q SPL, (q + 1) SPL) of a and b in registers (samples past n are zero
// padding up to whole 16-sample tiles), and every loop has compile-time
// bounds.  Sums over the samples (the codes E a, E b, E t, the per-pair norms,
// D^T r) are taken per lane and completed with DPP adds inside the group, in
// an order that leaves the same value on each of its lanes.  E, D and T are
// read from LDS, one address per lane of a group.  The sums over pairs of
// outer products,
//   dD = sum_p r_a' u^T + r_b' v^T + g_3 h^T,   dE = sum_p g_u a^T + g_v b^T + c_3 t^T
// (g_3 = g_S and c_3 = -w_code (2/k) d for Eq. 8; g_3 = lambda r_h and no third
// dE term for the two-term loss), are contractions over the pairs and run on
// the fp32 matrix cores (v_mfma_f32_16x16x4_f32, K = pairs).  For one term
// each lane writes its samples, as they are computed, down its pair's column
// of a per-wavefront [samples][pairs] LDS block; for the tile of samples
// 16c .. 16c+15, lane (g, m) reads row m, PPW/4 consecutive pairs (16- or
// 8-byte loads), one matrix step per pair.  Rows are PPW + 4 floats apart and
// the lane groups' row ranges start PPW banks apart, so the column writes fall
// on distinct banks, and so do the row reads of a lane group's rows.  The wavefronts of a
// workgroup are summed in a fixed order into one partial row.

template <int N>
struct LaneShape;
template <>
struct LaneShape<31> {
    static constexpr int NP = 32;       // samples padded to whole 16-sample tiles
    static constexpr int LPP = 2;       // lanes per pair
    static constexpr int THREADS = 512;
    static constexpr int XBLOCKS = 1;   // sample blocks per wavefront (1 or 2)
};

template <int N>
struct LaneDims : LaneShape<N> {
    using S = LaneShape<N>;
    static constexpr int SPL = S::NP / S::LPP;               // samples per lane
    static constexpr int PPW = kWave / S::LPP;               // pairs per wavefront
    static constexpr int WAVES = S::THREADS / kWave;
    static constexpr int PAIRS = WAVES * PPW;                // pairs per workgroup and chunk
    static constexpr int ROW = PPW + 4;                      // LDS row stride of the sample blocks
    // extra offset between consecutive lane groups' row ranges, so that they
    // start PPW banks apart
    static constexpr int QP = (((PPW - SPL * ROW) % 64) + 64) % 64;
    static constexpr int XSIZE = S::NP * ROW + (S::LPP - 1) * QP;
    static constexpr int NC = S::NP / 16;                    // 16-sample tiles
    static constexpr int STEPS = PPW / 4;                    // matrix steps per tile and term
    static_assert(S::NP % S::LPP == 0 && (STEPS == 2 || STEPS % 4 == 0), "lane shape");
};

typedef float hc_mf4 __attribute__((ext_vector_type(4)));

// Orders a wavefront's LDS writes before its later reads of other lanes'
// values (LDS executes one wavefront's instructions in order; this keeps the
// compiler from moving accesses across the point).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A compiler-level memory clobber: table reads from LDS after it are issued
// again instead of reusing (and keeping live) the values read before it.
__device__ __forceinline__ void reread_tables() { __asm__ volatile("" ::: "memory"); }

// x, opaque to the compiler: a product of it is recomputed where it is needed
// rather than kept in a register, and a finished sum is computed here rather
// than sunk towards a late use (which would keep its inputs live).
__device__ __forceinline__ float fresh(float x) {
    __asm__ volatile("" : "+v"(x));
    return x;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over the pair's LPP lanes (2, 4 or 8): pairwise, then pairs of pairs,
// then halves; every lane of the group ends with the same value.
template <int LPP>
__device__ __forceinline__ float pair_sum(float x) {
    x = x + dpp<0xB1>(x);                    // quad_perm 1,0,3,2: the xor-1 partner
    if (LPP >= 4) x = x + dpp<0x4E>(x);      // quad_perm 2,3,0,1: the xor-2 partner
    if (LPP == 8) x = x + dpp<0x141>(x);     // row_half_mirror: lane 7 - i of the eight
    return fresh(x);
}

// c += sum over the wave's PPW pairs of L[row m][pair] R[row m'][pair] for the
// 16 x 16 tile (m, m'); lrow / rrow point at pair STEPS g of the lane's rows.
typedef float hc_mf2 __attribute__((ext_vector_type(2)));

template <int STEPS>
__device__ __forceinline__ hc_mf4 contract(const float* lrow, const float* rrow, hc_mf4 c) {
    if (STEPS == 2) {
        const hc_mf2 x = *reinterpret_cast<const hc_mf2*>(lrow);
        const hc_mf2 y = *reinterpret_cast<const hc_mf2*>(rrow);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], y[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], y[1], c, 0, 0, 0);
        return c;
    }
#pragma unroll
    for (int v = 0; v < STEPS / 4; ++v) {
        const hc_mf4 x = *reinterpret_cast<const hc_mf4*>(lrow + 4 * v);
        const hc_mf4 y = *reinterpret_cast<const hc_mf4*>(rrow + 4 * v);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], y[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], y[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[2], y[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[3], y[3], c, 0, 0, 0);
    }
    return c;
}

template <bool EQ8, int K, int N>
__global__ __launch_bounds__(LaneShape<N>::THREADS) void codec_lanes_kernel(PartialArgs<float> a) {
    using L = LaneDims<N>;
    constexpr int NP = L::NP, LPP = L::LPP, SPL = L::SPL, PPW = L::PPW, ROW = L::ROW, QP = L::QP;
    constexpr int NC = L::NC, STEPS = L::STEPS, WAVES = L::WAVES, THREADS = L::THREADS;
    // D rows K4 + 2 floats apart: the rows SPL apart that a pair's lanes read
    // at once fall on different banks
    constexpr int DS = ((K + 3) & ~3) + 2;
    constexpr int TERMS_E = EQ8 ? 3 : 2;
    __shared__ __align__(16) float sE[K * NP];   // E, rows padded with 0
    __shared__ __align__(16) float sD[NP * DS];  // D, rows past n zero
    __shared__ __align__(16) float sT[3 * NP];
    __shared__ __align__(16) float sZero[PPW];
    __shared__ __align__(16) float sX[WAVES][L::XBLOCKS][L::XSIZE];  // [sample][pair]
    __shared__ __align__(16) float sY[WAVES][3 * K * ROW];          // [term][code][pair]
    __shared__ double s_loss[WAVES];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int pr = lane / LPP, q = lane % LPP;  // pair in the wave, lane in the pair
    const int i0 = SPL * q;                     // the lane's first sample
    const uint64_t ctr_base = a.draw ? draw_base(a) : 0ull;

    // the raw parameters and T this thread stages are loaded first, then the
    // first chunk's pair rows: loads complete in order, so the rows are still
    // in flight while the softplus values are formed and stored
    constexpr int IE = (K * NP + THREADS - 1) / THREADS, ID = (NP * DS + THREADS - 1) / THREADS;
    constexpr int IT = (3 * NP + THREADS - 1) / THREADS;
    // (indices clamped into the arrays, the values past them selected away)
    float rwe[IE], rwd[ID], rt[IT];
#pragma unroll
    for (int u = 0; u < IE; ++u) {
        const int e = min(tid + u * THREADS, K * NP - 1), j = e / NP, i = min(e % NP, N - 1);
        rwe[u] = a.we[j * N + i];
    }
#pragma unroll
    for (int u = 0; u < ID; ++u) {
        const int e = min(tid + u * THREADS, NP * DS - 1), i = min(e / DS, N - 1), j = min(e % DS, K - 1);
        rwd[u] = a.wd[i * K + j];
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
        const int e = min(tid + u * THREADS, 3 * NP - 1);
        rt[u] = EQ8 ? a.T[(e / NP) * N + min(e % NP, N - 1)] : 0.f;
    }
    const int last = N - 1 - i0;  // the lane's last sample below n, relative to i0
    // the lane's samples of a chunk's pair (row 0 for pairs past the batch);
    // samples past n re-read the last one (and are zeroed in the loop)
    float av[SPL], bv[SPL];
    auto load_rows = [&](int64_t ch) {
        const int64_t pi = ch * PPW + pr;
        int64_t ra = 0, rb = 0;
        if (pi < a.N) batch_rows(a, ctr_base, pi, ra, rb);
        const float* pa = a.A + ra * a.ld_a + i0;
        const float* pb = a.B + rb * a.ld_b + i0;
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int o = s < last ? s : last;
            av[s] = pa[o];
            bv[s] = pb[o];
        }
    };
    const int64_t ch0 = int64_t(blockIdx.x) * WAVES + wave;
    if (ch0 * PPW < a.N) load_rows(ch0);
#pragma unroll
    for (int u = 0; u < IE; ++u) {
        const int e = tid + u * THREADS, i = e % NP;
        if (e < K * NP) sE[e] = i < N ? softplus(rwe[u], a.beta) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < ID; ++u) {
        const int e = tid + u * THREADS, i = e / DS, j = e % DS;
        if (e < NP * DS) sD[e] = (i < N && j < K) ? softplus(rwd[u], a.beta) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
        const int e = tid + u * THREADS;
        if (EQ8 && e < 3 * NP) sT[e] = e % NP < N ? rt[u] : 0.f;
    }
    if (tid < PPW) sZero[tid] = 0.f;
    if (a.step && blockIdx.x == 0 && tid == 0) *a.ws_step = *a.step + 1;
    __syncthreads();

    const int g = lane >> 4, m = lane & 15;
    float* X0 = sX[wave][0];
    float* X1 = sX[wave][L::XBLOCKS - 1];
    float* Y = sY[wave];
    // the lane's columns: its sample s at xcol[s * ROW]
    const int col = i0 * ROW + q * QP + pr;
    float* xcol0 = X0 + col;
    float* xcol1 = X1 + col;
    float* ycol = Y + pr;
    // lane (g, m)'s row of the tile of samples 16c .. 16c+15
    auto xrow = [&](const float* X, int c) {
        const int i = 16 * c + m;
        return X + i * ROW + (i / SPL) * QP + STEPS * g;
    };
    // rows of the code blocks past k read zeros
    const float* yrow[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) yrow[t] = m < K ? Y + (t * K + m) * ROW + STEPS * g : sZero + STEPS * g;

    hc_mf4 gd[NC], ge[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) gd[c] = ge[c] = hc_mf4{0.f, 0.f, 0.f, 0.f};
    double loss_acc = 0.0;
    const float lam = a.lam;
    const float wr = EQ8 ? float(a.w_rec * 2.0 / N) : 1.f;
    const float wk = EQ8 ? float(a.w_code * 2.0 / K) : 0.f;

    for (int64_t ch = ch0; ch * PPW < a.N; ch += int64_t(gridDim.x) * WAVES) {
        // keeps the reads of E, D and T from LDS inside the loop: hoisted out
        // of it, all of them would stay live in registers
        reread_tables();
        if (ch != ch0) load_rows(ch);
        const bool valid = ch * PPW + pr < a.N;
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const bool in = valid && s <= last;
            av[s] = in ? av[s] : 0.f;
            bv[s] = in ? bv[s] : 0.f;
        }

        // codes u = E a, v = E b, h = u v (Eq. 4, Eq. 6); Eq. 8: d = h - E t,
        // with t = a b formed once per sample for this loop
        float u[K], v[K], h[K], dc[K];
        float tv[EQ8 ? SPL : 1];
        if (EQ8) {
#pragma unroll
            for (int s = 0; s < SPL; ++s) tv[EQ8 ? s : 0] = fresh(av[s]) * bv[s];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            float su = 0.f, sv = 0.f, sw = 0.f;
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                const float e = sE[j * NP + i0 + s];
                su = fmaf(e, av[s], su);
                sv = fmaf(e, bv[s], sv);
                if (EQ8) sw = fmaf(e, tv[EQ8 ? s : 0], sw);
            }
            u[j] = pair_sum<LPP>(su);
            v[j] = pair_sum<LPP>(sv);
            h[j] = u[j] * v[j];
            dc[j] = EQ8 ? fresh(h[j] - pair_sum<LPP>(sw)) : 0.f;
        }
        wave_lds_order();  // the previous chunk's reads of the blocks are done
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (q == t % LPP) {
#pragma unroll
                for (int j = 0; j < K; ++j) ycol[(t * K + j) * ROW] = t == 0 ? u[j] : (t == 1 ? v[j] : h[j]);
            }
        }

        // reconstructions D u, D v, D h of the lane's samples: the per-pair
        // sums, D^T r_a' and D^T r_b' accumulated as the residuals appear;
        // r_a' (and with two blocks r_b') written to the sample blocks
        reread_tables();
        float S[SPL], xb[L::XBLOCKS == 2 ? 1 : SPL];
        float gu[K], gv[K], gs[K];
#pragma unroll
        for (int j = 0; j < K; ++j) gu[j] = gv[j] = gs[j] = 0.f;
        float s_rr = 0.f, s_rh = 0.f, s_st = 0.f, s_ss = 0.f, s_tt = 0.f, s_c0 = 0.f, s_c1 = 0.f, s_c2 = 0.f;
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int i = i0 + s;  // rows of D and T past n are zero
            float du = 0.f, dv = 0.f, dh = 0.f;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const float d = sD[i * DS + j];
                du = fmaf(d, u[j], du);
                dv = fmaf(d, v[j], dv);
                dh = fmaf(d, h[j], dh);
            }
            const float ti = fresh(av[s]) * bv[s];
            const float rai = du - av[s], rbi = dv - bv[s], rh = dh - ti;
            S[s] = dh;
            s_rr = fmaf(rai, rai, fmaf(rbi, rbi, s_rr));
            s_rh = fmaf(rh, rh, s_rh);
            if (EQ8) {
                s_st = fmaf(dh, ti, s_st);
                s_ss = fmaf(dh, dh, s_ss);
                s_tt = fmaf(ti, ti, s_tt);
                s_c0 = fmaf(sT[i], rh, s_c0);
                s_c1 = fmaf(sT[NP + i], rh, s_c1);
                s_c2 = fmaf(sT[2 * NP + i], rh, s_c2);
            }
            // a pair past the batch has a = b = 0, so its residuals (and g_3
            // below: both norms clamp to eps, every factor stays finite) are 0
            const float rap = wr * rai, rbp = wr * rbi;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const float d = sD[i * DS + j];
                gu[j] = fmaf(d, rap, gu[j]);
                gv[j] = fmaf(d, rbp, gv[j]);
            }
            xcol0[s * ROW] = rap;
            if (L::XBLOCKS == 2)
                xcol1[s * ROW] = rbp;
            else
                xb[s] = rbp;
        }
        // dD terms r_a' u^T and r_b' v^T: rows = samples, columns = codes
        wave_lds_order();
#pragma unroll
        for (int c = 0; c < NC; ++c) gd[c] = contract<STEPS>(xrow(X0, c), yrow[0], gd[c]);
        if (L::XBLOCKS == 1) {
            wave_lds_order();
#pragma unroll
            for (int s = 0; s < SPL; ++s) xcol0[s * ROW] = xb[(L::XBLOCKS == 2) ? 0 : s];
            wave_lds_order();
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) gd[c] = contract<STEPS>(xrow(X1, c), yrow[1], gd[c]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            gu[j] = pair_sum<LPP>(gu[j]);
            gv[j] = pair_sum<LPP>(gv[j]);
        }
        s_rr = pair_sum<LPP>(s_rr);
        s_rh = pair_sum<LPP>(s_rh);
        if (EQ8) {
            s_st = pair_sum<LPP>(s_st);
            s_ss = pair_sum<LPP>(s_ss);
            s_tt = pair_sum<LPP>(s_tt);
            s_c0 = pair_sum<LPP>(s_c0);
            s_c1 = pair_sum<LPP>(s_c1);
            s_c2 = pair_sum<LPP>(s_c2);
        }

        // per-pair factors of the third term: g_3 = g_S (Eq. 8) or lambda r_h
        reread_tables();
        float al, bt, bs, g0 = 0.f, g1 = 0.f, g2 = 0.f;
        if (EQ8) {
            float s_dd = 0.f;
#pragma unroll
            for (int j = 0; j < K; ++j) s_dd = fmaf(dc[j], dc[j], s_dd);
            const double M = double(s_rh) / N;
            const double sn = sqrt(double(s_ss));
            const double ns = sn > a.eps ? sn : a.eps;
            const double tn = sqrt(double(s_tt));
            const double nt = tn > a.eps ? tn : a.eps;
            const double cs = double(s_st) / (ns * nt);
            if (valid && q == 0)
                loss_acc += a.w_e2e * M * (2.0 - cs) + a.w_rec * double(s_rr) / N + a.w_code * double(s_dd) / K +
                            a.w_col * (double(s_c0) * s_c0 + double(s_c1) * s_c1 + double(s_c2) * s_c2) / 3.0;
            // g_S = al r_h - bt t + bs S + T^T gc
            al = float(a.w_e2e * (2.0 - cs) * 2.0 / N);
            bt = float(a.w_e2e * M / (ns * nt));
            bs = float(sn > a.eps ? a.w_e2e * M * cs / double(s_ss) : 0.0);
            g0 = float(a.w_col * (2.0 / 3.0) * s_c0);
            g1 = float(a.w_col * (2.0 / 3.0) * s_c1);
            g2 = float(a.w_col * (2.0 / 3.0) * s_c2);
        } else {
            if (valid && q == 0) loss_acc += double(s_rr) + double(lam) * double(s_rh);
            al = lam;
            bt = 0.f;
            bs = 0.f;
        }
        wave_lds_order();  // the r_a' (r_b') tiles have been read
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int i = i0 + s;
            const float ti = fresh(av[s]) * bv[s];
            float g3 = al * (S[s] - ti) - bt * ti + bs * S[s];
            if (EQ8) g3 += g0 * sT[i] + g1 * sT[NP + i] + g2 * sT[2 * NP + i];
#pragma unroll
            for (int j = 0; j < K; ++j) gs[j] = fmaf(sD[i * DS + j], g3, gs[j]);
            xcol0[s * ROW] = g3;
        }
        // dD term g_3 h^T
        wave_lds_order();
#pragma unroll
        for (int c = 0; c < NC; ++c) gd[c] = contract<STEPS>(xrow(X0, c), yrow[2], gd[c]);
#pragma unroll
        for (int j = 0; j < K; ++j) gs[j] = pair_sum<LPP>(gs[j]);

        // code-space gradients g_u = D^T r_a' + g_h v, g_v = D^T r_b' + g_h u,
        // g_h = D^T g_3 (+ w_code (2/k) d for Eq. 8), then dE on the matrix
        // cores: rows = codes, columns = samples
        wave_lds_order();
#pragma unroll
        for (int t = 0; t < TERMS_E; ++t) {
            if (q == t % LPP) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const float dcp = (EQ8 && valid) ? wk * dc[j] : 0.f;
                    const float gh = gs[j] + dcp;
                    ycol[(t * K + j) * ROW] = t == 0 ? gu[j] + gh * v[j] : (t == 1 ? gv[j] + gh * u[j] : -dcp);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < TERMS_E; t += L::XBLOCKS) {
            if (t > 0) wave_lds_order();
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                xcol0[s * ROW] = t == 0 ? av[s] : (t == 1 ? bv[s] : fresh(av[s]) * bv[s]);
                if (L::XBLOCKS == 2 && t + 1 < TERMS_E) xcol1[s * ROW] = t == 0 ? bv[s] : fresh(av[s]) * bv[s];
            }
            wave_lds_order();
#pragma unroll
            for (int c = 0; c < NC; ++c) ge[c] = contract<STEPS>(yrow[t], xrow(X0, c), ge[c]);
            if (L::XBLOCKS == 2 && t + 1 < TERMS_E) {
#pragma unroll
                for (int c = 0; c < NC; ++c) ge[c] = contract<STEPS>(yrow[t + 1], xrow(X1, c), ge[c]);
            }
        }
    }

    // the wavefronts' tiles, then their fixed-order sum into the partial row;
    // [0, kn) is dL/dE (k x n), [kn, 2kn) dL/dD (n x k)
    constexpr int kn = K * N;
    static_assert(2 * kn <= L::XSIZE, "partial tile fits a sample block");
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * c + 4 * g + r, j = m;  // dD element of the tile
            if (i < N && j < K) X0[kn + i * K + j] = gd[c][r];
            const int j2 = 4 * g + r, i2 = 16 * c + m;  // dE element
            if (i2 < N && j2 < K) X0[j2 * N + i2] = ge[c][r];
        }
    }
    for (int mm = kWave / 2; mm >= 1; mm >>= 1) loss_acc += __shfl_xor(loss_acc, mm, kWave);
    if (lane == 0) s_loss[wave] = loss_acc;
    __syncthreads();
    double* prow = a.part + int64_t(blockIdx.x) * (2 * kn + 1);
    for (int e = tid; e < 2 * kn; e += THREADS) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) t += double(sX[w][0][e]);
        prow[e] = t;
    }
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < WAVES; ++w) t += s_loss[w];
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
    int64_t* step;  // Adam step counter: receives *ws_step
    double lr, beta1, beta2, eps;
    double ln_beta1, ln_beta2;
    int adam;
};

// One workgroup per 64 consecutive elements of the partial rows (lane l of
// every wavefront holds element 64 * block + l, so each row load is one
// coalesced 512-byte piece); its 16 wavefronts take every 16th row, sixteen
// loads in flight per lane, and their sums are added in wavefront order
// through LDS.  Wavefront 0 then applies the step to its 64 elements.
constexpr int kFinishWaves = 16;
constexpr int kFinishThreads = kFinishWaves * kWave;

template <typename F>
__global__ __launch_bounds__(kFinishThreads) void codec_finish_kernel(FinishArgs<F> a) {
    __shared__ double s_part[kFinishWaves][kWave];
    const int kn = a.k * a.n;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int e = blockIdx.x * kWave + lane;
    // the incremented step reaches the counter only now, after the pair draw
    // of this step has read it
    if (a.adam && blockIdx.x == 0 && threadIdx.x == 0) *a.step = *a.ws_step;
    const int64_t stride = 2 * kn + 1;
    const bool live = e <= 2 * kn;
    const bool isE = e < kn;
    const int idx = isE ? e : e - kn;
    F* w = isE ? a.we : a.wd;
    F* m = isE ? a.m_e : a.m_d;
    F* v = isE ? a.v_e : a.v_d;
    // wavefront 0's parameters, Adam state and step are fetched with the
    // partial rows, so their latency overlaps that of the sums
    double wt = 0.0, m0 = 0.0, v0 = 0.0, t = 0.0;
    if (wave == 0 && e < 2 * kn) {
        wt = double(w[idx]);
        if (a.adam) {
            m0 = double(m[idx]);
            v0 = double(v[idx]);
            t = double(*a.ws_step);
        }
    }
    // sixteen rows per lane in flight at once (256 rows in one round); rows
    // past the table add 0
    constexpr int kIlp = 16;
    double acc[kIlp];
#pragma unroll
    for (int u = 0; u < kIlp; ++u) {
        const int r = wave + u * kFinishWaves;
        acc[u] = live && r < a.rows ? a.part[int64_t(r) * stride + e] : 0.0;
    }
    // the step's bias corrections while the rows are in flight (beta^t =
    // exp(t ln beta), ln beta from the host)
    double bc1 = 1.0, bc2 = 1.0;
    if (a.adam && wave == 0) {
        bc1 = 1.0 - exp(t * a.ln_beta1);
        bc2 = 1.0 - exp(t * a.ln_beta2);
    }
    for (int r0 = wave + kIlp * kFinishWaves; r0 < a.rows; r0 += kIlp * kFinishWaves) {
        double x[kIlp];
#pragma unroll
        for (int u = 0; u < kIlp; ++u) {
            const int r = r0 + u * kFinishWaves;
            x[u] = live && r < a.rows ? a.part[int64_t(r) * stride + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kIlp; ++u) acc[u] += x[u];
    }
#pragma unroll
    for (int w2 = kIlp / 2; w2 >= 1; w2 >>= 1)
#pragma unroll
        for (int u = 0; u < w2; ++u) acc[u] += acc[u + w2];
    s_part[wave][lane] = acc[0];
    __syncthreads();
    if (wave != 0 || !live) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kFinishWaves; ++q) s += s_part[q][lane];
    if (e == 2 * kn) {
        *a.loss = F(s * a.inv_n);
        return;
    }
    const double g = s * a.gscale * slope(wt, a.beta);
    F* gout = isE ? a.grad_e : a.grad_d;
    if (gout) gout[idx] = F(g);
    if (a.adam) {
        const double mm = a.beta1 * m0 + (1.0 - a.beta1) * g;
        const double vv = a.beta2 * v0 + (1.0 - a.beta2) * g * g;
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

// ------------------------------------------------------------------ kernel 2, matrix-core tiles
//
// Float32 step for n = 81 with k <= 16: every product of the step is a
// 16x16x4 fp32 MFMA on tiles of 16 pairs, one wavefront per tile, eight
// wavefronts per workgroup (two per SIMD, so that one wavefront's matrix
// products overlap the other's LDS and vector work; no workgroup barrier
// inside the loop).  Per tile, with the pairs' spectra a, b in LDS as
// [pair][sample]:
//   codes        U = A E^T, V = B E^T, Tc = (A*B) E^T and P_a = A D,
//                P_b = B D, P_t = (A*B) D (pairs x codes, K = samples, one
//                pass over the spectra); H = U*V, Dc = H - Tc (Eq. 8's code
//                term);
//   residuals    A_hat = U D^T, B_hat = V D^T, S = H D^T (pairs x samples,
//                K = codes) minus a, b and t = a*b, summed per pair across
//                the lanes of a 16-lane row for the loss and the per-pair
//                factors of g_3, the gradient with respect to the decoded
//                product (Eq. 8: the cosine-scaled error, the colour term
//                through T);
//   code grads   with G = D^T D (k x k) the code-space gradients need no
//                pass over the samples: D^T r_a = U G - P_a, D^T r_b =
//                V G - P_b, D^T g_3 = al (H G - P_t) - bt P_t + bs H G +
//                sum_c gc_c (T_c D); then g_u = D^T r_a' + g_h v and
//                g_v = D^T r_b' + g_h u;
//   weight grads dD^T += U^T r_a' + V^T r_b' + H^T g_3 and dE += g_u^T A +
//                g_v^T B - w Dc^T (A*B) (codes x samples, K = the tile's
//                pairs), accumulated in registers across tiles.
// The contractions over the tile's pairs take both operands from registers:
// an MFMA output holds pair 4g + r of lane (g, n) in register r, which is
// the K index g of the product's r-th step.  So the residuals and the
// code-space gradients never pass through LDS; per wavefront LDS holds a,
// b and the [pair][code] tiles of U, V, H that the K = codes products read
// transposed.  The wavefronts' sums are added in a fixed order into one
// float64 partial row per workgroup.  Rows are read with a stride of 84
// floats (samples 81-83 zero; reads past sample 81 are clamped onto it),
// conflict-free for the 16 rows x 4 columns of a forward operand.
constexpr int kTileNS = 81;                 // samples
constexpr int kTileRS = 84;                 // LDS row stride of [pair][sample] tiles
constexpr int kTileKS = kTileRS / 4;        // K steps over the samples (21)
constexpr int kTileNB = 6;                  // 16-sample blocks (96 >= 81)
constexpr int kTileCS = 17;                 // row stride of [pair][code] and [code][code] tiles
constexpr int kTileWaves = 8;
constexpr int kTileThreads = kTileWaves * kWave;
constexpr int kTilePerWave = 2 * 16 * kTileRS + 3 * 16 * kTileCS;   // a, b; U, V, H
// E [16][RS], D [RS][CS], T [3][RS], G [16][CS], T D [3][16]
constexpr int kTileShared = 16 * kTileRS + kTileRS * kTileCS + 3 * kTileRS + 16 * kTileCS + 3 * 16;

size_t tile_lds_bytes() { return sizeof(float) * (size_t(kTileShared) + size_t(kTileWaves) * kTilePerWave); }

// 16-lane row sum (lanes n = 0..15 of one quarter) by data-parallel
// primitives within the row: the xor-1 and xor-2 partners, then lane 7 - i of
// the eight, then lane 15 - i of the sixteen.  Each step adds two equal-sized
// partial sums in either order, so every lane of the row ends with the same
// value.
__device__ __forceinline__ float row16_sum(float x) {
    x = x + dpp<0xB1>(x);                     // quad_perm 1,0,3,2
    x = x + dpp<0x4E>(x);                     // quad_perm 2,3,0,1
    x = x + dpp<0x141>(x);                    // row_half_mirror
    x = x + dpp<0x140>(x);                    // row_mirror
    return x;
}

// The value of quad lane Q (0..3), in every lane of each quad.
template <int Q>
__device__ __forceinline__ float quad_bcast(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), Q * 0x55, 0xF, 0xF, true));
}

// v[r] by selects on values (an index into the array would place it in
// private memory)
__device__ __forceinline__ float pick4(const float (&v)[4], int r) {
    const float x0 = v[0], x1 = v[1], x2 = v[2], x3 = v[3];
    const float lo = (r & 1) ? x1 : x0, hi = (r & 1) ? x3 : x2;
    return (r & 2) ? hi : lo;
}

__device__ __forceinline__ void quad_bcast4(float x, float (&v)[4]) {
    v[0] = quad_bcast<0>(x);
    v[1] = quad_bcast<1>(x);
    v[2] = quad_bcast<2>(x);
    v[3] = quad_bcast<3>(x);
}

template <bool EQ8, int K>
__global__ __launch_bounds__(kTileThreads) void codec_tile_kernel(PartialArgs<float> a) {
    extern __shared__ __align__(16) float tsm[];
    constexpr int NS = kTileNS, RS = kTileRS, CS = kTileCS, KS = kTileKS, NB = kTileNB;
    constexpr int KC = (K + 3) / 4;                   // K steps over the codes
    static_assert(K <= 16, "one 16-column block of codes");
    float* sE = tsm;                                  // [16 codes][RS], rows >= K zero
    float* sD = sE + 16 * RS;                         // [RS samples][CS], rows >= n and columns >= K zero
    float* sT = sD + RS * CS;                         // [3][RS]
    float* sG = sT + 3 * RS;                          // [16][CS]: G = D^T D
    float* sTD = sG + 16 * CS;                        // [3][16]: T D
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid & (kWave - 1), g = lane >> 4, n = lane & 15;
    float* XA = tsm + kTileShared + wave * kTilePerWave;
    float* XB = XA + 16 * RS;
    float* CU = XB + 16 * RS;                         // [pair][code] tiles
    float* CV = CU + 16 * CS;
    float* CH = CV + 16 * CS;

    for (int e = tid; e < 16 * RS; e += kTileThreads) {
        const int j = e / RS, i = e % RS;
        sE[e] = (j < K && i < NS) ? softplus(a.we[j * NS + i], a.beta) : 0.f;
    }
    for (int e = tid; e < RS * CS; e += kTileThreads) {
        const int i = e / CS, j = e % CS;
        sD[e] = (i < NS && j < K) ? softplus(a.wd[i * K + j], a.beta) : 0.f;
    }
    for (int e = tid; e < 3 * RS; e += kTileThreads) sT[e] = (EQ8 && e % RS < NS) ? a.T[(e / RS) * NS + e % RS] : 0.f;
    // samples 81..83 of the row tiles stay zero
    for (int e = lane; e < 2 * 16 * (RS - NS); e += kWave) {
        const int t = e / (16 * (RS - NS)), p = (e / (RS - NS)) % 16, i = NS + e % (RS - NS);
        XA[t * 16 * RS + p * RS + i] = 0.f;
    }
    if (a.step && blockIdx.x == 0 && tid == 0) *a.ws_step = *a.step + 1;
    __syncthreads();
    // G = D^T D and T D: each entry one thread's sum over the samples in order
    if (tid < 256) {
        const int j = tid >> 4, j2 = tid & 15;
        float s = 0.f;
        for (int i = 0; i < NS; ++i) s = fmaf(sD[i * CS + j], sD[i * CS + j2], s);
        sG[j * CS + j2] = s;
    } else if (tid < 256 + 48) {
        const int c = (tid - 256) >> 4, j = tid & 15;
        float s = 0.f;
        for (int i = 0; i < NS; ++i) s = fmaf(sT[c * RS + i], sD[i * CS + j], s);
        sTD[c * 16 + j] = s;
    }
    __syncthreads();

    const uint64_t ctr_base = a.draw ? draw_base(a) : 0ull;
    const float lam = a.lam;
    const float wr = EQ8 ? float(a.w_rec * 2.0 / NS) : 1.f;
    const float wk = EQ8 ? float(a.w_code * 2.0 / K) : 0.f;
    const float td0 = EQ8 ? sTD[n] : 0.f, td1 = EQ8 ? sTD[16 + n] : 0.f, td2 = EQ8 ? sTD[32 + n] : 0.f;
    hc_mf4 accD[NB], accE[NB];                        // dD^T and dE: code 4g + r, sample 16b + n
#pragma unroll
    for (int b = 0; b < NB; ++b) accD[b] = accE[b] = hc_mf4{0.f, 0.f, 0.f, 0.f};
    double loss_acc = 0.0;
    // the tile's rows are loaded with lane l taking pair l / 4 of the tile and
    // its samples q, q + 4, q + 8, ... with q = l % 4
    const int lp = lane >> 2, lq = lane & 3;
    constexpr int PER = (NS + 3) / 4;                 // 21 samples per lane and row
    const int64_t tiles = (a.N + 15) / 16;
    const int64_t tstride = int64_t(gridDim.x) * kTileWaves;
    // the rows of a tile (pairs past N read zeros); the next tile's are
    // loaded during the current tile's last phase
    float va[PER], vb[PER];
    auto load_rows = [&](int64_t t) {
        const int64_t pi = t * 16 + lp;
        int64_t ra = 0, rb = 0;
        const bool ok = t < tiles && pi < a.N;
        if (ok) batch_rows(a, ctr_base, pi, ra, rb);
        const float* pa = a.A + ra * a.ld_a;
        const float* pb = a.B + rb * a.ld_b;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = lq + 4 * u;
            va[u] = (ok && i < NS) ? pa[i] : 0.f;
            vb[u] = (ok && i < NS) ? pb[i] : 0.f;
        }
    };
    load_rows(int64_t(blockIdx.x) * kTileWaves + wave);
    for (int64_t tile = int64_t(blockIdx.x) * kTileWaves + wave; tile < tiles; tile += tstride) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = lq + 4 * u;
            if (i < NS) {
                XA[lp * RS + i] = va[u];
                XB[lp * RS + i] = vb[u];
            }
        }
        wave_lds_order();
        // ---- codes and the spectra's projections on D (pairs x codes), K = samples
        hc_mf4 cu = {0.f, 0.f, 0.f, 0.f}, cv = cu, ct = cu, pa = cu, pb = cu, pt = cu;
#pragma unroll 3
        for (int st = 0; st < KS; ++st) {
            const int i = 4 * st + g;
            const float e = sE[n * RS + i], d = sD[i * CS + n];
            const float xa = XA[n * RS + i], xb = XB[n * RS + i], xt = xa * xb;
            cu = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, e, cu, 0, 0, 0);
            cv = __builtin_amdgcn_mfma_f32_16x16x4f32(xb, e, cv, 0, 0, 0);
            if (EQ8) ct = __builtin_amdgcn_mfma_f32_16x16x4f32(xt, e, ct, 0, 0, 0);
            pa = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, d, pa, 0, 0, 0);
            pb = __builtin_amdgcn_mfma_f32_16x16x4f32(xb, d, pb, 0, 0, 0);
            pt = __builtin_amdgcn_mfma_f32_16x16x4f32(xt, d, pt, 0, 0, 0);
        }
        // lane (g, n): pairs 4g + r, code n; the code term's loss is added here
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 4 * g + r;
            const float h = cu[r] * cv[r];
            const float dc = EQ8 ? h - ct[r] : 0.f;
            CU[p * CS + n] = cu[r];
            CV[p * CS + n] = cv[r];
            CH[p * CS + n] = h;
            if (EQ8) {
                const float dd = row16_sum(n < K ? dc * dc : 0.f);
                if (n == 0 && tile * 16 + p < a.N) loss_acc += a.w_code * double(dd) * (1.0 / K);
            }
            ct[r] = dc;                               // kept for g_h
        }
        wave_lds_order();
        // ---- the codes as [pair n][code 4st + g] operands; U G - P_a, V G - P_b,
        // H G (pairs x codes, K = codes)
        float cuT[KC], cvT[KC], chT[KC];
        hc_mf4 ug = -pa, vg = -pb, hg = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < KC; ++st) {
            const int j = 4 * st + g;
            cuT[st] = CU[n * CS + j];
            cvT[st] = CV[n * CS + j];
            chT[st] = CH[n * CS + j];
            const float gv = sG[j * CS + n];
            ug = __builtin_amdgcn_mfma_f32_16x16x4f32(cuT[st], gv, ug, 0, 0, 0);
            vg = __builtin_amdgcn_mfma_f32_16x16x4f32(cvT[st], gv, vg, 0, 0, 0);
            hg = __builtin_amdgcn_mfma_f32_16x16x4f32(chT[st], gv, hg, 0, 0, 0);
        }
        // S.S = sum_j H_j (H G)_j and S.t = sum_j H_j (t D)_j per pair (sums of
        // non-negative terms), for lane n's pair 4g + (n & 3)
        const int rq = n & 3;
        float q_ss = 0.f, q_st = 0.f;
        if (EQ8) {
            float x_ss[4], x_st[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float h = cu[r] * cv[r];
                x_ss[r] = row16_sum(h * hg[r]);
                x_st[r] = row16_sum(h * pt[r]);
            }
            q_ss = pick4(x_ss, rq);
            q_st = pick4(x_st, rq);
        }
        // ---- reconstructions and residuals per 16-sample block; r_a' and r_b'
        // go straight into dD^T, S is kept for g_3
        float s_rr[4] = {0.f, 0.f, 0.f, 0.f}, s_rh[4] = {0.f, 0.f, 0.f, 0.f}, s_tt[4] = {0.f, 0.f, 0.f, 0.f};
        float s_c0[4] = {0.f, 0.f, 0.f, 0.f}, s_c1[4] = {0.f, 0.f, 0.f, 0.f}, s_c2[4] = {0.f, 0.f, 0.f, 0.f};
        hc_mf4 sh[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            hc_mf4 ra = {0.f, 0.f, 0.f, 0.f}, rb = ra;
            sh[b] = ra;
            const int i = 16 * b + n;                 // the lane's sample of the block
            // past the samples, reads land on sample 81, zero in every tile
            const int ic = i < NS ? i : NS;
#pragma unroll
            for (int st = 0; st < KC; ++st) {
                const float d = sD[ic * CS + 4 * st + g];
                ra = __builtin_amdgcn_mfma_f32_16x16x4f32(cuT[st], d, ra, 0, 0, 0);
                rb = __builtin_amdgcn_mfma_f32_16x16x4f32(cvT[st], d, rb, 0, 0, 0);
                sh[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(chT[st], d, sh[b], 0, 0, 0);
            }
            const float t0 = EQ8 ? sT[ic] : 0.f, t1 = EQ8 ? sT[RS + ic] : 0.f, t2 = EQ8 ? sT[2 * RS + ic] : 0.f;
            float r1[4], r2[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 4 * g + r;
                const float av = XA[p * RS + ic], bv = XB[p * RS + ic];
                const float ti = av * bv;
                // zero past the samples: the reconstruction and the spectrum both are
                const float rai = ra[r] - av, rbi = rb[r] - bv, rh = sh[b][r] - ti;
                r1[r] = wr * rai;
                r2[r] = wr * rbi;
                s_rr[r] = fmaf(rai, rai, fmaf(rbi, rbi, s_rr[r]));
                s_rh[r] = fmaf(rh, rh, s_rh[r]);
                if (EQ8) {
                    s_tt[r] = fmaf(ti, ti, s_tt[r]);
                    s_c0[r] = fmaf(t0, rh, s_c0[r]);
                    s_c1[r] = fmaf(t1, rh, s_c1[r]);
                    s_c2[r] = fmaf(t2, rh, s_c2[r]);
                }
            }
            // dD^T (codes x the block's samples) += U^T r_a' + V^T r_b', K = pairs
#pragma unroll
            for (int r = 0; r < 4; ++r) accD[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cu[r], r1[r], accD[b], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) accD[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[r], r2[r], accD[b], 0, 0, 0);
        }
        // per-pair sums across the 16 lanes of the row; lane n then takes the
        // factors of pair 4g + (n & 3) alone, and each quad shares them
        float rr, rhh, tt = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
        {
            float x[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = row16_sum(s_rr[r]);
            rr = pick4(x, rq);
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = row16_sum(s_rh[r]);
            rhh = pick4(x, rq);
            if (EQ8) {
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = row16_sum(s_tt[r]);
                tt = pick4(x, rq);
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = row16_sum(s_c0[r]);
                c0 = pick4(x, rq);
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = row16_sum(s_c1[r]);
                c1 = pick4(x, rq);
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = row16_sum(s_c2[r]);
                c2 = pick4(x, rq);
            }
        }
        const bool own = n < 4 && tile * 16 + 4 * g + rq < a.N;    // one lane adds each pair's loss
        // g_3 = fs S - ft t + sum_c gc_c T_c (fs = al + bs, ft = al + bt)
        float f_s, f_t, f_c0 = 0.f, f_c1 = 0.f, f_c2 = 0.f;
        if (EQ8) {
            const double M = double(rhh) * (1.0 / NS);
            const double sn = sqrt(double(q_ss));
            const double ns = sn > a.eps ? sn : a.eps;
            const double tn = sqrt(double(tt));
            const double nt = tn > a.eps ? tn : a.eps;
            const double inv_nn = 1.0 / (ns * nt);
            const double cs = double(q_st) * inv_nn;
            if (own)
                loss_acc += a.w_e2e * M * (2.0 - cs) + a.w_rec * double(rr) * (1.0 / NS) +
                            a.w_col * (double(c0) * c0 + double(c1) * c1 + double(c2) * c2) * (1.0 / 3.0);
            const double al = a.w_e2e * (2.0 - cs) * (2.0 / NS);
            const double bt = a.w_e2e * M * inv_nn;
            const double bs = sn > a.eps ? a.w_e2e * M * cs / double(q_ss) : 0.0;
            f_s = float(al + bs);
            f_t = float(al + bt);
            f_c0 = float(a.w_col * (2.0 / 3.0) * c0);
            f_c1 = float(a.w_col * (2.0 / 3.0) * c1);
            f_c2 = float(a.w_col * (2.0 / 3.0) * c2);
        } else {
            if (own) loss_acc += double(rr) + double(lam) * double(rhh);
            f_s = f_t = lam;
        }
        float fs[4], ft[4], gc0[4] = {0.f, 0.f, 0.f, 0.f}, gc1[4] = {0.f, 0.f, 0.f, 0.f};
        float gc2[4] = {0.f, 0.f, 0.f, 0.f};
        quad_bcast4(f_s, fs);
        quad_bcast4(f_t, ft);
        if (EQ8) {
            quad_bcast4(f_c0, gc0);
            quad_bcast4(f_c1, gc1);
            quad_bcast4(f_c2, gc2);
        }
        // ---- code-space gradients (pair 4g + r, code n) through G
        float cgu[4], cgv[4], cdc[4];
        {
            const float td0 = EQ8 ? sTD[n] : 0.f, td1 = EQ8 ? sTD[16 + n] : 0.f, td2 = EQ8 ? sTD[32 + n] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float gh = fs[r] * hg[r] - ft[r] * pt[r];
                if (EQ8) gh += (gc0[r] * td0 + gc1[r] * td1 + gc2[r] * td2) + wk * ct[r];
                cgu[r] = wr * ug[r] + gh * cv[r];
                cgv[r] = wr * vg[r] + gh * cu[r];
                cdc[r] = -wk * ct[r];
            }
        }
        // ---- g_3 (pair 4g + r, sample 16b + n) into dD^T += H^T g_3
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = 16 * b + n, ic = i < NS ? i : NS;
            const float t0 = EQ8 ? sT[ic] : 0.f, t1 = EQ8 ? sT[RS + ic] : 0.f, t2 = EQ8 ? sT[2 * RS + ic] : 0.f;
            float g3[4];                              // zero past the samples: S, t and T all are
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 4 * g + r;
                const float ti = XA[p * RS + ic] * XB[p * RS + ic];
                g3[r] = fs[r] * sh[b][r] - ft[r] * ti;
                if (EQ8) g3[r] += gc0[r] * t0 + gc1[r] * t1 + gc2[r] * t2;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) accD[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cu[r] * cv[r], g3[r], accD[b], 0, 0, 0);
        }
        load_rows(tile + tstride);
        // ---- dE += g_u^T A + g_v^T B - w Dc^T (A*B), K = the tile's pairs
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = 16 * b + n, ic = i < NS ? i : NS;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 4 * g + r;
                const float xa = XA[p * RS + ic], xb = XB[p * RS + ic];
                accE[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cgu[r], xa, accE[b], 0, 0, 0);
                accE[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cgv[r], xb, accE[b], 0, 0, 0);
                if (EQ8) accE[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(cdc[r], xa * xb, accE[b], 0, 0, 0);
            }
        }
        wave_lds_order();   // the tiles are read before the next tile's rows land
    }

    // ---- the wavefronts' sums into the partial row, in a fixed order:
    // [0, kn) dL/dE (k x n), [kn, 2kn) dL/dD (n x k)
    constexpr int kn = K * NS;
    static_assert(kTileWaves * 2 * kn <= kTileWaves * kTilePerWave, "scratch fits the wave tiles");
    __shared__ double s_loss[kTileWaves];
    for (int mm = kWave / 2; mm >= 1; mm >>= 1) loss_acc += __shfl_xor(loss_acc, mm, kWave);
    __syncthreads();
    float* scr = tsm + kTileShared + wave * 2 * kn;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = 4 * g + r, i = 16 * b + n;          // code j, sample i
            if (j < K && i < NS) {
                scr[j * NS + i] = accE[b][r];
                scr[kn + i * K + j] = accD[b][r];
            }
        }
    }
    if (lane == 0) s_loss[wave] = loss_acc;
    __syncthreads();
    double* prow = a.part + int64_t(blockIdx.x) * (2 * kn + 1);
    for (int e = tid; e < 2 * kn; e += kTileThreads) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kTileWaves; ++w) t += double(tsm[kTileShared + w * 2 * kn + e]);
        prow[e] = t;
    }
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kTileWaves; ++w) t += s_loss[w];
        prow[2 * kn] = t;
    }
}

// float64 never takes the few-lanes-per-pair kernel (`lanes` is false for it);
// this overload only lets run<double> compile.
inline void launch_lanes(const PartialArgs<double>&, bool, int, int, int64_t, hipStream_t) {}

template <int N>
void launch_lanes_n(const PartialArgs<float>& p, bool eq8, int k, int64_t rows, hipStream_t st) {
    const dim3 grid(static_cast<uint32_t>(rows)), block(LaneShape<N>::THREADS);
    if (k == 6) {
        if (eq8) hipLaunchKernelGGL((codec_lanes_kernel<true, 6, N>), grid, block, 0, st, p);
        else hipLaunchKernelGGL((codec_lanes_kernel<false, 6, N>), grid, block, 0, st, p);
    } else {
        if (eq8) hipLaunchKernelGGL((codec_lanes_kernel<true, 9, N>), grid, block, 0, st, p);
        else hipLaunchKernelGGL((codec_lanes_kernel<false, 9, N>), grid, block, 0, st, p);
    }
}

inline void launch_lanes(const PartialArgs<float>& p, bool eq8, int k, int, int64_t rows, hipStream_t st) {
    launch_lanes_n<31>(p, eq8, k, rows, st);
}

// float64 never takes the tile kernel; this overload only lets run<double> compile.
inline void launch_tiles(const PartialArgs<double>&, bool, int, int64_t, hipStream_t) {}

inline void launch_tiles(const PartialArgs<float>& p, bool eq8, int k, int64_t rows, hipStream_t st) {
    const dim3 grid(static_cast<uint32_t>(rows)), block(kTileThreads);
    const size_t lds = tile_lds_bytes();
    if (k == 6) {
        if (eq8) hipLaunchKernelGGL((codec_tile_kernel<true, 6>), grid, block, lds, st, p);
        else hipLaunchKernelGGL((codec_tile_kernel<false, 6>), grid, block, lds, st, p);
    } else {
        if (eq8) hipLaunchKernelGGL((codec_tile_kernel<true, 9>), grid, block, lds, st, p);
        else hipLaunchKernelGGL((codec_tile_kernel<false, 9>), grid, block, lds, st, p);
    }
}

// Pairs per workgroup of the few-lanes-per-pair kernel (n = 31).
inline int64_t lane_pairs(int) { return LaneDims<31>::PAIRS; }

// float32 at n = 81 with k = 6 or 9 takes the matrix-core tile kernel, at
// n = 31 the few-lanes-per-pair kernel (one partial row per 256 pairs); both
// stage softplus(Wt) themselves
template <typename F>
bool takes_tiles(int k, int n) {
    return std::is_same<F, float>::value && n == kTileNS && (k == 6 || k == 9);
}

template <typename F>
bool takes_lanes(int k, int n) {
    return std::is_same<F, float>::value && n == 31 && (k == 6 || k == 9);
}

constexpr int64_t kTileGrid = 256;   // workgroups of the tile kernel (one per CU)

// Partial rows (workgroups of the partials kernel) of a step.
template <typename F>
int64_t step_rows(const hc_codec_args& a) {
    if (takes_tiles<F>(a.k, a.n)) return std::min<int64_t>(ceil_div(ceil_div(a.N, 16), kTileWaves), kTileGrid);
    return takes_lanes<F>(a.k, a.n) ? std::min<int64_t>(ceil_div(a.N, lane_pairs(a.n)), kMaxRows)
                                    : plan(a.k, a.n, a.N, sizeof(F), a.objective).grid;
}

// Workspace bytes a step uses (the layout of carve).
template <typename F>
size_t step_workspace(const hc_codec_args& a) {
    const size_t kn = size_t(a.k) * a.n;
    return 2 * align8(kn * sizeof(F)) + size_t(step_rows<F>(a)) * (2 * kn + 1) * sizeof(double) +
           sizeof(int64_t);
}

template <typename F>
hc_status run(const hc_codec_args& a) {
    const int k = a.k, n = a.n, kn = k * n;
    hipStream_t st = reinterpret_cast<hipStream_t>(a.stream);
    const bool eq8 = a.objective == HC_CODEC_EQ8;
    const Plan pl = plan(k, n, a.N, sizeof(F), a.objective);
    const bool tiles = takes_tiles<F>(k, n);
    const bool lanes = takes_lanes<F>(k, n);
    const int64_t rows = step_rows<F>(a);
    Workspace ws = carve(a.workspace, k, n, rows, sizeof(F));
    int64_t* adam_step = a.adam ? a.adam->step : nullptr;
    hc_status s = HC_OK;
    if (!lanes && !tiles && !pl.ed_in_lds) {
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
    p.draw = a.draw != nullptr;
    p.key_a = a.draw ? stream_key(a.draw->seed_a, kIndexStream) : 0;
    p.key_b = a.draw ? stream_key(a.draw->seed_b, kIndexStream) : 0;
    p.draw_ctr0 = a.draw ? a.draw->ctr0 : 0;
    p.draw_scale = a.draw ? a.draw->ctr_scale_dev : nullptr;
    p.N = a.N;
    p.n_tiles = pl.n_tiles;
    p.part = ws.part;
    p.ed_in_lds = pl.ed_in_lds;
    p.we = static_cast<const F*>(a.Wt_E);
    p.wd = static_cast<const F*>(a.Wt_D);
    p.beta = F(a.beta);
    p.step = (lanes || tiles || pl.ed_in_lds) ? adam_step : nullptr;
    p.ws_step = ws.step;
    p.T = static_cast<const F*>(a.T);
    p.w_e2e = a.w_e2e;
    p.w_rec = a.w_rec;
    p.w_code = a.w_code;
    p.w_col = a.w_col;
    p.eps = a.cos_eps;
    if (tiles)
        launch_tiles(p, eq8, k, rows, st);
    else if (lanes)
        launch_lanes(p, eq8, k, n, rows, st);
    else if (eq8)
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
    f.rows = int(rows);
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
        // beta = 0 gives exp(t * -inf) = 0 for every step t >= 1
        f.ln_beta1 = std::log(a.adam->beta1);
        f.ln_beta2 = std::log(a.adam->beta2);
    } else {
        f.m_e = f.v_e = f.m_d = f.v_d = nullptr;
        f.lr = f.beta1 = f.beta2 = f.eps = 0.0;
        f.ln_beta1 = f.ln_beta2 = 0.0;
    }
    f.ws_step = ws.step;
    f.step = adam_step;
    const int g2 = int(ceil_div(2 * kn + 1, kWave));
    hipLaunchKernelGGL(codec_finish_kernel<F>, dim3(g2), dim3(kFinishThreads), 0, st, f);
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

// ------------------------------------------------------------------ step without allocation
//
// Scratch of hc_codec_step_static: a device array the code object brings
// with it, so the entry point never allocates.  Each device holds its own
// copy at its own address, obtained once per device with
// hipGetSymbolAddress; host code uses only those addresses (the array's name
// in host code is a host-side stand-in, not a device address).

static __device__ __align__(256) unsigned char scratch[HC_CODEC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of the scratch array, or NULL (error
// set) if it cannot be obtained.
void* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("hc_codec_step_static: no current HIP device (or device index >= %d)", kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("hc_codec_step_static: hipGetSymbolAddress of the scratch array failed on device %d: %s",
                      dev, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

size_t codec_static_need(const hc_codec_args& a) {
    return a.dtype == 1 ? step_workspace<double>(a) : step_workspace<float>(a);
}

hc_status launch_codec_step_static(const hc_codec_args& a) {
    const size_t need = codec_static_need(a);
    if (need > size_t(HC_CODEC_STATIC_SCRATCH_BYTES)) {
        set_error("hc_codec_step_static: this shape needs %zu bytes of scratch, above the %zu of the "
                  "static array",
                  need, size_t(HC_CODEC_STATIC_SCRATCH_BYTES));
        return HC_ENOMEM;
    }
    void* ws = scratch_address();
    if (ws == nullptr) return HC_EDEVICE;
    // every partial row, weight and step slot the kernels read is written
    // earlier in the same step, so nothing needs clearing between calls
    hc_codec_args b = a;
    b.workspace = ws;
    b.workspace_bytes = size_t(HC_CODEC_STATIC_SCRATCH_BYTES);
    return launch_codec_step(b);
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
