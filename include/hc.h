/*
 * hc.h -- C ABI of the Hadamard-code light-path library (gfx950 / MI355X).
 *
 * Spectral rendering multiplies n-sample spectra element-wise along light
 * paths and integrates the result against colour-matching functions.  The
 * Hadamard-code method (Yu, Guarnera, Guarnera, "Compact Hadamard Latent
 * Codes for Efficient Spectral Rendering", arXiv 2602.18741) replaces the
 * n samples by k = 3B non-negative linear codes z = W_enc s (Eq. 4), takes
 * the element-wise product block by block on B RGB-style triplets (Eq. 6),
 * and decodes once per frame with W_dec and the colour-matching matrix.
 * This library evaluates both forms for batches of light paths on one GPU.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns hc_status.  HC_OK (0) means the work was enqueued.
 *   On any other status nothing was enqueued and hc_last_error() returns a
 *   thread-local description of the first problem found.
 * - Pointers are device pointers unless stated otherwise.  The caller owns
 *   and allocates every buffer; the library never allocates, frees or keeps a
 *   pointer past the return of the call.  Scratch memory is passed in as an
 *   explicit workspace.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  The
 *   calls only enqueue work on it; there is no implicit synchronisation.
 *   Faults inside kernels surface at the caller's next synchronisation.
 * - float4 data (spectra rows, code rows, latent images) needs 16-byte aligned
 *   base pointers and row strides (ld) that are multiples of 4 floats.
 * - Latent rows use the blocked "RGBx" layout: code channel c lives at float
 *   offset 4*(c/3) + c%3 of its row, so block b (channels 3b..3b+2, one RGB
 *   pass of Sec. 6.1) is the 16-byte slot [4b, 4b+4) and its 4th float is 0.
 *   A row of a k-channel code therefore needs ld >= 4*ceil(k/3) floats.  A k
 *   that is not a multiple of 3 is treated as k padded with zero channels.
 * - Limits: 1 <= n <= 128 spectral samples, 1 <= k <= 48 code channels,
 *   spp >= 1, path length 0..255, light id < 2^24, fewer than 2^32 vertex
 *   records and texels per call.
 */
#ifndef HC_H
#define HC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hc_status;
#define HC_OK 0
#define HC_EINVAL 1       /* null pointer or invalid scalar argument */
#define HC_ESHAPE 2       /* sizes or strides out of the supported range */
#define HC_EALIGN 3       /* pointer or stride misaligned */
#define HC_ENOMEM 4       /* workspace too small */
#define HC_EDEVICE 5      /* a HIP call or kernel launch failed */
#define HC_EUNSUPPORTED 6 /* valid request outside the compiled kernel variants */

/* Name of a status code ("HC_OK", ...).  Static string, never NULL. */
const char* hc_status_string(hc_status s);
/* Description of the last error on the calling thread ("" if none).  Valid
 * until the next hc_* call on the same thread. */
const char* hc_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t hc_version(void);

/*
 * Light-path records (a host struct holding device pointers).
 * Paths are pixel-major: pixel q owns paths [q*spp, (q+1)*spp).
 *   hdr[p]        uint32: light id in bits 0-23, number of reflectance
 *                 vertices L_p (0..255) in bits 24-31.  L_p = 0 means the
 *                 path sees the light directly.
 *   pix_first[q]  uint32: index of pixel q's first vertex record.  A pixel's
 *                 paths store their vertices back to back, in path order.
 *   vtx[2*j]      uint32 texel (or material) index of vertex record j,
 *   vtx[2*j+1]    IEEE-754 bits of its float32 weight.  8-byte aligned.
 * Records outside the assets (texel >= n_texels, light >= n_illum) are
 * clamped to the last valid index and vertex records at or past n_vertices
 * are skipped, so that no read leaves the buffers; the value computed for
 * such a pixel is unspecified.  hc_check_paths detects them.
 */
typedef struct hc_paths {
    int64_t n_pixels;
    int32_t spp;
    int32_t reserved0;
    const uint32_t* hdr;
    const uint32_t* pix_first;
    const uint32_t* vtx;
    int64_t n_vertices;
} hc_paths;

/* Spectral assets: reflectance rows refl[t*ld + i] (n_texels x n, i < n) and
 * light rows illum[l*ld_illum + i] (n_illum x n).  float32, 16-byte aligned,
 * ld and ld_illum multiples of 4 and >= n; ld < 2^30 (a row stride below
 * 4 GiB). */
typedef struct hc_spectral_assets {
    const float* refl;
    int64_t n_texels;
    int32_t n;
    int32_t reserved0;
    int64_t ld;
    const float* illum;
    int32_t n_illum;
    int32_t reserved1;
    int64_t ld_illum;
} hc_spectral_assets;

/* Latent assets: encoded texels codes[t*ld + ...] and encoded lights
 * illum_codes[l*ld_illum + ...] in the blocked RGBx layout, k channels;
 * ld < 2^31. */
typedef struct hc_latent_assets {
    const float* codes;
    int64_t n_texels;
    int32_t k;
    int32_t reserved0;
    int64_t ld;
    const float* illum_codes;
    int32_t n_illum;
    int32_t reserved1;
    int64_t ld_illum;
} hc_latent_assets;

/*
 * hc_encode -- linear encoder z = W_enc s of Eq. 4, applied to m spectra.
 *   E  : k x n row-major float32 (W_enc, non-negative in the method).
 *   S  : m rows of n float32 samples, row stride ld_s floats.
 *   Z  : m latent rows (blocked RGBx layout), row stride ld_z >= 4*ceil(k/3).
 *        Every float of Z[i, 0:ld_z) is written; pad positions get 0.
 * Used once per asset (textures, materials and lights are encoded once,
 * Fig. 2b).
 */
hc_status hc_encode(const float* E, int32_t k, int32_t n, const float* S, int64_t m,
                    int64_t ld_s, float* Z, int64_t ld_z, void* stream);

/*
 * hc_shade_spectral -- plain spectral form.  For each path p of pixel q:
 *   S_p = light_{id_p} * prod_{v < L_p} (w_{p,v} * refl_{t_{p,v}})   (element-wise
 *   products over n samples: the scale and multiply operations of Sec. 3),
 *   x_p = T S_p (T = T_cmf, 3 x n row-major float32, quadrature folded in),
 *   xyz[q] = (1/spp) sum_{p in q} x_p.
 *   xyz: n_pixels x 3 float32, contiguous.
 */
hc_status hc_shade_spectral(const hc_paths* paths, const hc_spectral_assets* assets,
                            const float* T, float* xyz, void* stream);

/*
 * hc_shade_latent -- latent form (Eq. 6 blockwise products, Sec. 6.1 passes).
 * For each path p of pixel q and code block b in [block_first,
 * block_first + block_count):
 *   Z_p^(b) = code(light_{id_p})^(b) (.) prod_{v < L_p} (w_{p,v} * code(t_{p,v})^(b)),
 *   zimg[q]^(b) = (1/spp) sum_{p in q} Z_p^(b)
 * written to the 16-byte slot b of row q of zimg (row stride ld_zimg floats;
 * the slot's 4th float is written 0; other slots are untouched).
 * block_count = ceil(k/3) with block_first = 0 is the fused call; a call per
 * block is one "RGB pass", and the passes re-assemble into the same image.
 * Each channel's arithmetic does not depend on the blocks in the call, so
 * fused and per-pass images are bitwise equal.
 */
hc_status hc_shade_latent(const hc_paths* paths, const hc_latent_assets* assets,
                          int32_t block_first, int32_t block_count, float* zimg,
                          int64_t ld_zimg, void* stream);

/*
 * hc_decode_xyz -- decode a latent image once per frame (Eq. 4, right; Fig. 2b).
 *   D: n x k row-major float32 (W_dec).  T: 3 x n row-major float32.
 *   zimg: n_pixels latent rows (blocked layout), stride ld_zimg.
 *   xyz[q] = T (D z_q), n_pixels x 3 contiguous float32.
 *   spectra (nullable): spectra[q*ld_spectra + i] = (D z_q)_i for i < n;
 *   ld_spectra >= n (any alignment of 4 bytes).
 */
hc_status hc_decode_xyz(const float* D, int32_t n, int32_t k, const float* T,
                        const float* zimg, int64_t n_pixels, int64_t ld_zimg, float* xyz,
                        float* spectra, int64_t ld_spectra, void* stream);

/*
 * hc_decode_matrix -- the per-pixel decode of Eq. 4 (right) as one matrix,
 * M = T D, so that xyz = M z for a latent pixel z.
 *   D: n x k row-major float32 (W_dec).  T: 3 x n row-major float32.
 *   M: 3 rows of 3*ceil(k/3) float32, row-major, columns in the blocked
 *      channel order of the latent layout (channel c of block b at column
 *      3b + c); the columns past k are written 0.  Caller-owned, 4-byte
 *      aligned.
 * Entry (r, c) is summed over the n samples in order; hc_decode_xyz stages
 * the same entries, so an image decoded by either route has the same bits.
 */
hc_status hc_decode_matrix(const float* D, int32_t n, int32_t k, const float* T, float* M,
                           void* stream);

/*
 * hc_shade_latent_xyz -- the latent frame in one launch (Eq. 6 products over
 * all ceil(k/3) blocks, Sec. 6.1, then the per-pixel decode of Eq. 4 / Fig. 2b):
 *   xyz[q] = M zimg[q],
 * where zimg[q] is the pixel mean hc_shade_latent computes (not stored) and
 * M comes from hc_decode_matrix.  xyz: n_pixels x 3 float32, contiguous,
 * 4-byte aligned.  The result equals hc_shade_latent (all blocks) followed by
 * hc_decode_xyz with the D and T that gave M, bit for bit.  Shape, record
 * and alignment requirements are those of hc_shade_latent.
 */
hc_status hc_shade_latent_xyz(const hc_paths* paths, const hc_latent_assets* assets, const float* M,
                              float* xyz, void* stream);

/*
 * hc_check_paths -- count invalid records (see hc_paths).
 *   counts: 3 device uint64: [0] paths whose light id >= n_illum,
 *   [1] vertex records (counted once per pixel range covering them) whose
 *   texel >= n_texels, [2] pixels whose records run past n_vertices (their
 *   vertices are not examined).  The call overwrites counts.
 */
hc_status hc_check_paths(const hc_paths* paths, int64_t n_texels, int32_t n_illum,
                         uint64_t* counts, void* stream);

/*
 * Table-driven launches for serving many frames at once.
 *
 * A frame table entry describes one frame in either form: its records (as
 * hc_paths), its texture (`tex`: latent codes in the blocked layout, or
 * spectral rows) and light table (`lights`: light codes or light spectra),
 * the latent image it writes (latent form only) and its n_pixels x 3 XYZ
 * output.  A tile names a frame and a pixel range [begin, end).  The tables
 * and the tile / job counts live in device memory, so a captured HIP graph
 * can replay the same launches with new contents; each launch runs a fixed
 * grid of `grid` workgroups that walk the table (grid <= 65536; grid <= 0
 * lets the library take twice the number of the kernel's workgroups the
 * device holds at once).  Tile entries whose frame
 * index is out of [0, n_frames) are skipped and pixel ranges are clipped to
 * the frame; the frame entries themselves must satisfy the preconditions of
 * hc_shade_latent / hc_shade_spectral (they are not checked on the device).
 * Per-pixel results equal those of the single-frame calls bit for bit: a
 * pixel's samples are reduced inside one wavefront in the same order.
 */
typedef struct hc_frame {
    const uint32_t* hdr;
    const uint32_t* pix_first;
    const uint32_t* vtx;
    int64_t n_pixels;
    int64_t n_vertices;
    int32_t spp;
    int32_t n_illum;
    const float* tex;
    int64_t n_texels;
    int64_t ld_tex;     /* < 2^31 for codes, < 2^30 for spectral rows */
    const float* lights;
    int64_t ld_lights;
    float* image;       /* latent image rows (latent form), stride ld_image */
    int64_t ld_image;
    float* xyz;         /* n_pixels x 3 */
} hc_frame;

typedef struct hc_tile {
    int32_t frame;
    int32_t reserved0;
    int64_t begin;
    int64_t end;
} hc_tile;

/* Latent shading (all B blocks fused) of the tiles; k shared by all frames. */
hc_status hc_shade_latent_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                                const int32_t* n_tiles, int32_t max_tiles, int32_t k, int32_t grid,
                                void* stream);
/* Latent shading of the tiles with the per-pixel decode in the epilogue (as
 * hc_shade_latent_xyz): the tiles' pixels of frame xyz, with one decoder
 * matrix M (hc_decode_matrix, 3 x 3*ceil(k/3)) for every frame; the frames'
 * latent images are neither read nor written.  Bit for bit equal to
 * hc_shade_latent_tiles followed by hc_decode_tiles with the D and T of M. */
hc_status hc_shade_latent_xyz_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                                    const int32_t* n_tiles, int32_t max_tiles, int32_t k, const float* M,
                                    int32_t grid, void* stream);
/* Spectral shading of the tiles (n samples, T = T_cmf 3 x n) into frame xyz. */
hc_status hc_shade_spectral_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                                  const int32_t* n_tiles, int32_t max_tiles, int32_t n,
                                  const float* T, int32_t grid, void* stream);
/* Decode of the tiles' latent pixels to XYZ with one codec (as hc_decode_xyz). */
hc_status hc_decode_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                          const int32_t* n_tiles, int32_t max_tiles, const float* D, int32_t n,
                          int32_t k, const float* T, int32_t grid, void* stream);

/* Encode of many spectra arrays with one encoder (as hc_encode, rows
 * [begin, end) of S into Z); jobs and n_jobs in device memory. */
typedef struct hc_encode_job {
    const float* S;
    float* Z;
    int64_t ld_s;
    int64_t ld_z;
    int64_t begin;
    int64_t end;
} hc_encode_job;

hc_status hc_encode_jobs(const hc_encode_job* jobs, const int32_t* n_jobs, int32_t max_jobs,
                         const float* E, int32_t k, int32_t n, int32_t grid, void* stream);

/*
 * Codec fitting (Sec. 4.3 objectives with softplus weights, Eq. 5).
 *
 * Parameters Wt_E (k x n) and Wt_D (n x k), row-major; the codec is
 * E = softplus_beta(Wt_E), D = softplus_beta(Wt_D).  On a batch of N pairs
 * (a_i, b_i), with u = E a, v = E b, h = u (.) v (blockwise product, Eq. 6),
 * S_hat = D h and t = a * b, the objective is one of:
 *
 * HC_CODEC_L2 (objective 0):
 *   L = (1/N) sum_i ( |D u - a|^2 + |D v - b|^2 + lambda |S_hat - t|^2 ),
 *   the reconstruction term L_rec plus lambda times the squared-error part of
 *   L_e2e, squared norms summed over the n samples.
 * HC_CODEC_EQ8 (objective 1), the weighted four-term loss of Eq. 8, every
 *   MSE a mean over a pair's elements and then over the batch:
 *   L = w_e2e mean_i[ MSE(S_hat, t) (2 - cos(S_hat, t)) ]
 *     + w_rec (MSE(D u, a) + MSE(D v, b)) + w_code MSE(h, E t)
 *     + w_col MSE(T S_hat, T t),
 *   cos(x, y) = x.y / (max(|x|, cos_eps) max(|y|, cos_eps)); T is the 3 x n
 *   colour-matching matrix (dtype below).  The paper's weights are
 *   (0.5, 0.75, 1.0, 0.5) (Sec. 4.5).
 *
 * The call writes L and, if requested, dL/dWt_E and dL/dWt_D (hand-derived
 * backward), and optionally applies one Adam step.
 *
 * dtype: 0 = float32 everywhere, 1 = float64 everywhere (parameters, data,
 * T, outputs, Adam state).  Gradient sums run in that precision over tiles of
 * at most 64 pairs and in float64 across tiles, in a fixed order, so results
 * are deterministic.  (float32 with n = 31 or 81 and k = 6 or 9 spreads each
 * pair over 2 or 8 lanes and sums each wavefront's pairs on the fp32 matrix
 * cores: 32 or 8 pairs per wavefront and chunk, in float32 over the chunks a
 * wavefront takes - one each up to N = 262,144 (n = 31) or 65,536 (n = 81) -
 * and in float64 across wavefronts.)
 * Batch rows: row i of the a-batch is A[idx_a[i]*ld_a ...] when idx_a is
 * not NULL, else A[i*ld_a ...]; likewise b.  Indices must be < rows_a
 * (rows_b); out-of-range indices are clamped.  With draw not NULL the rows
 * are drawn on the device instead (idx_a and idx_b must then be NULL): row i
 * of the a-batch is the index hc_gen_indices(draw->seed_a, draw->ctr0,
 * draw->ctr_scale_dev, N, rows_a, ...) writes at position i, likewise b with
 * seed_b, so a fitting loop needs no index arrays and no extra launches.
 * When ctr_scale_dev is the Adam step counter, the draw sees its value from
 * before the call (the counter is incremented by the call's last kernel).
 */
#define HC_CODEC_L2 0
#define HC_CODEC_EQ8 1

typedef struct hc_adam {
    void* m_E;          /* k x n first moments (dtype) */
    void* v_E;          /* k x n second moments */
    void* m_D;          /* n x k */
    void* v_D;
    int64_t* step;      /* device counter: steps taken; incremented by the call */
    double lr, beta1, beta2, eps;
} hc_adam;

typedef struct hc_pair_draw {
    uint64_t seed_a, seed_b;
    uint64_t ctr0;
    const int64_t* ctr_scale_dev;  /* device counter, nullable */
} hc_pair_draw;

typedef struct hc_codec_args {
    int32_t k, n;
    int32_t dtype;
    int32_t objective;  /* HC_CODEC_L2 or HC_CODEC_EQ8 */
    double beta;        /* softplus sharpness (10 in the paper) */
    double lambda;      /* HC_CODEC_L2: weight of the product term */
    void* Wt_E;         /* updated in place when adam != NULL */
    void* Wt_D;
    const void* A;
    const void* B;
    int64_t ld_a, ld_b; /* row strides in elements */
    int64_t rows_a, rows_b;
    const uint32_t* idx_a;  /* nullable */
    const uint32_t* idx_b;  /* nullable */
    int64_t N;          /* batch size, >= 1 */
    void* loss;         /* device scalar (dtype) */
    void* grad_E;       /* nullable, k x n */
    void* grad_D;       /* nullable, n x k */
    const hc_adam* adam;    /* host pointer, nullable */
    void* workspace;
    size_t workspace_bytes;
    void* stream;
    /* HC_CODEC_EQ8 only (ignored otherwise): */
    const void* T;      /* 3 x n, row-major */
    double w_e2e, w_rec, w_code, w_col;  /* finite, >= 0 */
    double cos_eps;     /* > 0; 1e-8 is customary */
    const hc_pair_draw* draw;  /* host pointer, nullable: batch rows drawn on the device */
} hc_codec_args;

/* Bytes of workspace hc_codec_step needs for this shape, for either
 * objective (8-byte aligned). */
size_t hc_codec_workspace_size(int32_t k, int32_t n, int64_t N);
hc_status hc_codec_step(const hc_codec_args* args);

/*
 * hc_codec_step without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results
 * as hc_codec_step, except that args->workspace must be NULL and
 * args->workspace_bytes 0: the scratch is a static device array of
 * HC_CODEC_STATIC_SCRATCH_BYTES (16 MiB) that each GPU the library runs on
 * holds until the process ends (its address is looked up once per device,
 * on the first call there).  A shape whose step needs more scratch than
 * that (for example float64 with large k x n) is refused with HC_ENOMEM;
 * float32 steps of the fitting recipe (N = 65,536, n <= 81, k <= 9) fit.
 * Calls on one GPU share its array, and each call writes every value of it
 * that it reads before reading it: calls that overlap on one GPU (on
 * different streams, or from different host threads) race and must be
 * serialised by the caller.  No device memory is allocated or freed.
 */
#define HC_CODEC_STATIC_SCRATCH_BYTES (16u << 20)
hc_status hc_codec_step_static(const hc_codec_args* args);

/* E = softplus_beta(Wt_E), D = softplus_beta(Wt_D) as float32 (Eq. 5); the
 * matrices hc_encode and hc_decode_xyz take.  dtype of Wt_* as above. */
hc_status hc_codec_weights(const void* Wt_E, const void* Wt_D, int32_t k, int32_t n,
                           int32_t dtype, double beta, float* E, float* D, void* stream);

/*
 * RGB-to-latent upsampling network (Sec. 5): for each of m texels with linear
 * RGB colour c (row i of rgb, 3 floats, row stride ld_rgb >= 3),
 *   z = W3 silu(W2 silu(W1 c + b1) + b2) + b3,  silu(x) = x / (1 + exp(-x)),
 * hidden width 128 (three fully connected layers, Sec. 5.1), written to Z in
 * the blocked RGBx code layout of hc_encode (ld_z >= 4 ceil(k/3); padding
 * written as 0), ready for hc_shade_latent.  All weights are float32,
 * row-major device arrays: W1 128 x 3, b1 128, W2 128 x 128, b2 128,
 * W3 k x 128, b3 k (1 <= k <= 48).
 *
 * precision HC_MLP_F32: fp32 matrix-core products (v_mfma_f32_16x16x4_f32),
 * fp32 activations.  HC_MLP_F16: the 128 x 128 and output layers take fp16
 * operands (weights and activations rounded to fp16) with fp32
 * accumulation on the fp16 matrix cores; layer 1 and the activations stay
 * fp32.  The weights are read once per workgroup; rgb and Z are streamed.
 * m = 0 enqueues nothing.
 */
#define HC_MLP_F32 0
#define HC_MLP_F16 1

typedef struct hc_mlp {
    int32_t k;          /* output channels */
    int32_t hidden;     /* must be 128 */
    const float* W1;
    const float* b1;
    const float* W2;
    const float* b2;
    const float* W3;
    const float* b3;
} hc_mlp;

hc_status hc_upsample(const hc_mlp* net, int32_t precision, const float* rgb, int64_t m,
                      int64_t ld_rgb, float* Z, int64_t ld_z, void* stream);

/*
 * Training step of the upsampling network (Sec. 5.2).  Parameters are one
 * packed float32 array of hc_upsample_param_count(k, 128) values: W1 (128 x 3),
 * b1 (128), W2 (128 x 128), b2 (128), W3 (k x 128), b3 (k), in this order.
 * On a batch of N samples (colour c_i = rgb row idx[i], target code z_gt row
 * idx[i] in the blocked layout; rows 0..N-1 when idx is NULL; indices >= rows
 * are clamped) the loss is
 *   L = (1/N) sum_i [ |z_i - z_gt,i|^2 / k + w_max max_c |z_ic - z_gt,ic|
 *                     + w_col DeltaE76(Lab(M z_i), Lab(M z_gt,i)) ],
 * z_i the network output, M = T D (3 x k, float32: XYZ of a code through the
 * frozen decoder), Lab against the reference white (Xn, Yn, Zn).  The paper
 * uses w_max = 0.3 and w_col = 0.05.  The call writes L (device float) and,
 * if grad is not NULL, dL/dparams (hand-derived backward; at a tie of the
 * largest |z - z_gt| the first channel takes the max term's gradient).
 * With opt it then clips the gradient to the global L2 norm max_grad_norm
 * (factor min(1, max_grad_norm / (norm + 1e-6))), applies decoupled weight
 * decay (params *= 1 - lr weight_decay) and the Adam update with bias
 * correction, and increments *opt->step (AdamW with clipping, Sec. 5.2).
 * Deterministic.  workspace: hc_upsample_train_workspace_size(k, N) bytes,
 * 256-byte aligned.  Batch rows: idx[i] (clamped below rows) when idx is not
 * NULL, else i; with draw not NULL they are drawn on the device instead (idx
 * must then be NULL): sample i is row hc_gen_indices(draw->seed, draw->ctr0,
 * draw->ctr_scale_dev, N, rows, ...)[i].  When ctr_scale_dev is the
 * optimizer's step counter, the draw sees its value from before the call.
 */
typedef struct hc_index_draw {
    uint64_t seed;
    uint64_t ctr0;
    const int64_t* ctr_scale_dev;  /* device counter, nullable */
} hc_index_draw;

typedef struct hc_adamw {
    float* m;           /* first moments, packed like the parameters */
    float* v;           /* second moments */
    int64_t* step;      /* device counter */
    double lr, beta1, beta2, eps, weight_decay, max_grad_norm;
} hc_adamw;

typedef struct hc_upsample_train_args {
    int32_t k;
    int32_t hidden;     /* must be 128 */
    float* params;      /* updated in place when opt != NULL */
    const float* rgb;
    int64_t ld_rgb;     /* >= 3 */
    const float* z_gt;
    int64_t ld_z;       /* >= 4 ceil(k/3) */
    int64_t rows;       /* rows of rgb and z_gt */
    const uint32_t* idx;  /* nullable */
    int64_t N;          /* batch size, >= 1 */
    const float* M;     /* 3 x k */
    double white[3];
    double w_max, w_col;
    float* loss;        /* device scalar */
    float* grad;        /* nullable */
    const hc_adamw* opt;  /* host pointer, nullable */
    void* workspace;
    size_t workspace_bytes;
    void* stream;
    const hc_index_draw* draw;  /* host pointer, nullable: batch rows drawn on the device */
} hc_upsample_train_args;

int64_t hc_upsample_param_count(int32_t k, int32_t hidden);
size_t hc_upsample_train_workspace_size(int32_t k, int64_t N);
hc_status hc_upsample_train_step(const hc_upsample_train_args* args);

/*
 * Synthetic light-path generator (workload input, not part of the method).
 * Draws come from SplitMix64's output function mix64 applied to
 * key + (counter + 1) * 0x9E3779B97F4A7C15 with key = mix64(mix64(seed) + stream):
 *   path p (stream 1): r = rand(p); L = l_min + ((r & 0xFFFFFFFF) * (l_max-l_min+1) >> 32);
 *                      light = (r >> 32) * n_illum >> 32
 *   vertex v of path p (stream 2): r = rand(p*256 + v);
 *                      texel = (r & 0xFFFFFFFF) * n_tex >> 32; weight = (r >> 40) * 2^-24
 * Two steps: hc_gen_path_headers writes hdr, pix_first and the total vertex
 * count (device uint64); the caller reads the total, allocates vtx and calls
 * hc_gen_path_vertices.  workspace: hc_gen_workspace_size(n_pixels) bytes.
 */
typedef struct hc_path_gen {
    int64_t n_pixels;
    int32_t spp;
    int32_t l_min, l_max;
    int32_t n_illum;
    int64_t n_tex;
    uint64_t seed;
} hc_path_gen;

size_t hc_gen_workspace_size(int64_t n_pixels);
hc_status hc_gen_path_headers(const hc_path_gen* g, uint32_t* hdr, uint32_t* pix_first,
                              uint64_t* n_vertices, void* workspace, size_t workspace_bytes,
                              void* stream);
hc_status hc_gen_path_vertices(const hc_path_gen* g, const uint32_t* pix_first, uint32_t* vtx,
                               int64_t n_vertices, void* stream);
/* count indices uniform in [0, n) at counters ctr0 + i of stream 3 of seed;
 * if ctr_scale_dev is not NULL the counter base is ctr0 + (*ctr_scale_dev) * count
 * (a device step counter, so a captured graph draws new indices per replay). */
hc_status hc_gen_indices(uint64_t seed, uint64_t ctr0, const int64_t* ctr_scale_dev,
                         int64_t count, int64_t n, uint32_t* out, void* stream);

/*
 * Random-gather probe (measurement, not part of the method).  Reads every
 * vertex record of vtx (uint32 pairs {texel, float bits of the weight}, as
 * in hc_paths) and the first 4 * ceil(row_floats / 4) floats (whole 16-byte
 * chunks, as the shading kernels load rows) of row texel of table (row
 * stride ld floats; texels past n_rows are clamped to the last row), and
 * adds weight * (sum of those floats) into a per-lane sum; each of the
 * grid * 256 lanes writes its sum to out[lane].  The shading kernels gather
 * the same rows for the same records, so this rate, with nothing else done,
 * bounds theirs: for uniformly random texels each row costs whole cache
 * lines and the rate is the memory system's random-line rate, not its
 * streaming bandwidth.
 *   unroll          1, 2, 4 or 8 vertices in flight per lane (or lane group);
 *   lanes_per_row   1 (one lane loads the whole row, row_floats <= 16) or
 *                   8 (the row's 16-byte chunks over 8 lanes, <= 128 floats);
 *   grid            workgroups of 256 lanes (>= 1); out holds grid * 256 floats.
 * table, vtx and out need 16-, 8- and 4-byte alignment, ld a multiple of 4.
 */
hc_status hc_gather_probe(const uint32_t* vtx, int64_t n_vertices, const float* table, int64_t n_rows,
                          int64_t ld, int32_t row_floats, int32_t unroll, int32_t lanes_per_row,
                          int32_t grid, float* out, void* stream);

/*
 * Streaming probe (measurement, not part of the method): the device's
 * sequential bandwidth, the reference the gather rates and the streaming
 * kernels (encode, decode) are compared with.  src holds n16 16-byte chunks.
 *   mode 0 (read)  every chunk is read and its four floats added into a
 *                  per-lane sum; each of the grid * 256 lanes writes its sum
 *                  to dst[lane] (dst holds grid * 256 floats, 4-byte aligned);
 *   mode 1 (copy)  the chunks are copied to dst (n16 chunks, 16-byte aligned).
 *   grid           workgroups of 256 lanes, [1, 2^20]; chunks are taken in a
 *                  grid-stride loop, four per lane in flight.
 * src needs 16-byte alignment; n16 in [0, 2^40).
 */
hc_status hc_stream_probe(const float* src, float* dst, int64_t n16, int32_t mode, int32_t grid, void* stream);

/*
 * Issue-rate probe (measurement, not part of the method): the cost of single
 * vector instructions, the reference for a kernel bound by its arithmetic
 * issue (the upsampling network's activation: an exponential and a
 * reciprocal per value).  Each of the grid * 256 lanes runs
 * HC_ALU_PROBE_CHAINS independent chains of HC_ALU_PROBE_ITERS applications
 * of one instruction, then writes the sum of its chains to out[lane] (out
 * holds grid * 256 floats, 4-byte aligned; the values carry no meaning).
 *   op  0 fp32 multiply-add, 1 v_exp_f32, 2 v_rcp_f32, 3 v_exp_f16,
 *       4 v_rcp_f16, 5 packed fp16 multiply-add (two values an instruction);
 *   grid  workgroups of 256 lanes (4 wavefronts), [1, 2^20].
 * Time the launch on the stream: cycles per wavefront instruction per SIMD =
 * seconds * clock * SIMDs / (grid * 4 * chains * iters).
 */
#define HC_ALU_PROBE_CHAINS 8
#define HC_ALU_PROBE_ITERS 2048
hc_status hc_alu_probe(int32_t op, float* out, int32_t grid, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
