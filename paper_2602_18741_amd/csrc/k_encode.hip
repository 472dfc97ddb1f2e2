// Linear encode z = E s (per texel / material / light) and per-pixel decode
// xyz = (T D) z, optionally s_hat = D z.  Both are tiny contractions (k x n
// with k <= 48, n <= 128) done in registers against matrices staged in LDS;
// the kernels stream rows, so HBM bandwidth bounds them.

#include "hc_internal.hpp"

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
    int rows;        // rows per block (256 / 128 / 64)
};

// Block: stage `rows` spectra (coalesced float4 loads) and E in LDS, then one
// thread per row accumulates the k codes over the n samples in order.
template <int NB>
__global__ __launch_bounds__(kThreads) void encode_kernel(EncodeArgs a) {
    extern __shared__ float smem[];
    const int stride = 4 * a.nq + 1;  // odd stride: a thread's row reads hit distinct banks
    float* s_rows = smem;
    float* s_E = smem + a.rows * stride;
    const int tid = threadIdx.x;
    for (int i = tid; i < 3 * NB * a.n; i += kThreads) s_E[i] = (i < a.k * a.n) ? a.E[i] : 0.f;
    const int64_t r0 = int64_t(blockIdx.x) * a.rows;
    const int nrows = int(min<int64_t>(a.rows, a.m - r0));
    for (int i = tid; i < nrows * a.nq; i += kThreads) {
        const int r = i / a.nq, c = i % a.nq;
        const float4 v = ld4(a.S + (r0 + r) * a.ld_s + 4 * c);
        float* d = s_rows + r * stride + 4 * c;
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
    }
    __syncthreads();
    if (tid >= nrows) return;
    const float* s = s_rows + tid * stride;
    // channels past k read zero rows of E (staged that way), so they stay 0
    float z[3 * NB];
#pragma unroll
    for (int c = 0; c < 3 * NB; ++c) z[c] = 0.f;
    for (int i = 0; i < a.n; ++i) {
        const float si = s[i];
#pragma unroll
        for (int c = 0; c < 3 * NB; ++c) z[c] += s_E[c * a.n + i] * si;
    }
    float* out = a.Z + (r0 + tid) * a.ld_z;
#pragma unroll
    for (int b = 0; b < NB; ++b) st4(out + 4 * b, make_float4(z[3 * b], z[3 * b + 1], z[3 * b + 2], 0.f));
    for (int64_t f = 4 * NB; f < a.ld_z; f += 4) st4(out + f, make_float4(0.f, 0.f, 0.f, 0.f));
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

// One thread per pixel.  Each block first forms M = T D (3 x k) in LDS.
template <int NB>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeArgs a) {
    __shared__ float s_M[3 * kMaxK];
    extern __shared__ float s_D[];  // n x k, only when spectra are requested
    const int tid = threadIdx.x;
    for (int e = tid; e < 9 * NB; e += kThreads) {
        const int ch = e / (3 * NB), c = e % (3 * NB);
        float acc = 0.f;
        if (c < a.k)
            for (int i = 0; i < a.n; ++i) acc += a.T[ch * a.n + i] * a.D[i * a.k + c];
        s_M[e] = acc;
    }
    if (a.spectra)
        for (int e = tid; e < a.n * a.k; e += kThreads) s_D[e] = a.D[e];
    __syncthreads();
    const int64_t q = int64_t(blockIdx.x) * kThreads + tid;
    if (q >= a.n_pixels) return;
    float z[3 * NB];
    const float* row = a.zimg + q * a.ld_z;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float4 v = ld4(row + 4 * b);
        z[3 * b] = v.x;
        z[3 * b + 1] = v.y;
        z[3 * b + 2] = v.z;
    }
    // M has zero columns past k (see above), so padded channels add nothing
    float x = 0.f, y = 0.f, w = 0.f;
#pragma unroll
    for (int c = 0; c < 3 * NB; ++c) {
        x += s_M[c] * z[c];
        y += s_M[3 * NB + c] * z[c];
        w += s_M[6 * NB + c] * z[c];
    }
    float* o = a.xyz + q * 3;
    o[0] = x;
    o[1] = y;
    o[2] = w;
    if (a.spectra) {
        float* sp = a.spectra + q * a.ld_s;
        for (int i = 0; i < a.n; ++i) {
            float acc = 0.f;
            for (int c = 0; c < a.k; ++c) acc += s_D[i * a.k + c] * z[c];
            sp[i] = acc;
        }
    }
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
    a.rows = a.nq <= 8 ? 256 : (a.nq <= 16 ? 128 : 64);
    const int nb = (k + 2) / 3;
    const size_t lds = (size_t(a.rows) * (4 * a.nq + 1) + size_t(3 * nb) * n) * sizeof(float);
    const uint32_t blocks = uint32_t(ceil_div(m, a.rows));
    switch (nb) {
#define HC_ENC(NB) \
    case NB: hipLaunchKernelGGL(encode_kernel<NB>, dim3(blocks), dim3(kThreads), lds, st, a); break;
        HC_ENC(1) HC_ENC(2) HC_ENC(3) HC_ENC(4) HC_ENC(5) HC_ENC(6) HC_ENC(7) HC_ENC(8)
        HC_ENC(9) HC_ENC(10) HC_ENC(11) HC_ENC(12) HC_ENC(13) HC_ENC(14) HC_ENC(15) HC_ENC(16)
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
    const int64_t blocks = ceil_div(n_pixels, kThreads);
    if (blocks > 0x7FFFFFFF) {
        set_error("hc_decode_xyz: too many pixels for one launch");
        return HC_ESHAPE;
    }
    switch (a.nb) {
#define HC_DEC(NB)                                                                               \
    case NB:                                                                                     \
        hipLaunchKernelGGL(decode_kernel<NB>, dim3(uint32_t(blocks)), dim3(kThreads), lds, st, a); \
        break;
        HC_DEC(1) HC_DEC(2) HC_DEC(3) HC_DEC(4) HC_DEC(5) HC_DEC(6) HC_DEC(7) HC_DEC(8)
        HC_DEC(9) HC_DEC(10) HC_DEC(11) HC_DEC(12) HC_DEC(13) HC_DEC(14) HC_DEC(15) HC_DEC(16)
#undef HC_DEC
        default:
            set_error("hc_decode_xyz: k=%d unsupported", k);
            return HC_EUNSUPPORTED;
    }
    return launch_status("hc_decode_xyz");
}

}  // namespace hc
