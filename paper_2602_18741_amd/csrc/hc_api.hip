// C ABI entry points: argument validation, then the launchers.
// Nothing is enqueued unless every check passes.

#include <cstdarg>
#include <cstring>

#include "hc_internal.hpp"

namespace hc {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

hc_status launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: launch failed: %s", what, hipGetErrorString(e));
        return HC_EDEVICE;
    }
    return HC_OK;
}

// the issue-rate probe (k_probe.hip); a measurement only, so declared here
// rather than with the path's launchers
hc_status launch_alu_probe(int op, float* out, int grid, hipStream_t st);

}  // namespace hc

using namespace hc;

#define HC_REQUIRE(cond, code, ...)  \
    do {                             \
        if (!(cond)) {               \
            set_error(__VA_ARGS__);  \
            return (code);           \
        }                            \
    } while (0)

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

hc_status check_paths_struct(const hc_paths* P, const char* fn) {
    HC_REQUIRE(P != nullptr, HC_EINVAL, "%s: paths is NULL", fn);
    HC_REQUIRE(P->n_pixels >= 0, HC_ESHAPE, "%s: n_pixels < 0", fn);
    HC_REQUIRE(P->spp >= 1, HC_ESHAPE, "%s: spp must be >= 1 (got %d)", fn, P->spp);
    HC_REQUIRE(P->n_vertices >= 0 && P->n_vertices < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_vertices must be in [0, 2^32)", fn);
    HC_REQUIRE(P->n_pixels <= (int64_t(1) << 40) / P->spp, HC_ESHAPE, "%s: too many paths", fn);
    if (P->n_pixels > 0) {
        HC_REQUIRE(P->hdr && P->pix_first, HC_EINVAL, "%s: hdr/pix_first is NULL", fn);
        HC_REQUIRE(aligned4(P->hdr) && aligned4(P->pix_first), HC_EALIGN,
                   "%s: hdr/pix_first must be 4-byte aligned", fn);
    }
    if (P->n_vertices > 0) {
        HC_REQUIRE(P->vtx != nullptr, HC_EINVAL, "%s: vtx is NULL", fn);
        HC_REQUIRE(aligned8(P->vtx), HC_EALIGN, "%s: vtx must be 8-byte aligned", fn);
    }
    return HC_OK;
}

}  // namespace

extern "C" {

const char* hc_status_string(hc_status s) {
    switch (s) {
        case HC_OK: return "HC_OK";
        case HC_EINVAL: return "HC_EINVAL";
        case HC_ESHAPE: return "HC_ESHAPE";
        case HC_EALIGN: return "HC_EALIGN";
        case HC_ENOMEM: return "HC_ENOMEM";
        case HC_EDEVICE: return "HC_EDEVICE";
        case HC_EUNSUPPORTED: return "HC_EUNSUPPORTED";
        default: return "HC_UNKNOWN";
    }
}

const char* hc_last_error(void) { return g_err; }

int32_t hc_version(void) { return 100; }

hc_status hc_encode(const float* E, int32_t k, int32_t n, const float* S, int64_t m, int64_t ld_s,
                    float* Z, int64_t ld_z, void* stream) {
    clear_error();
    const char* fn = "hc_encode";
    HC_REQUIRE(k >= 1 && k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, k, kMaxK);
    HC_REQUIRE(n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: n=%d outside [1, %d]", fn, n, kMaxN);
    HC_REQUIRE(m >= 0 && m < (int64_t(1) << 32), HC_ESHAPE, "%s: m outside [0, 2^32)", fn);
    const int64_t nb = ceil_div(k, 3);
    HC_REQUIRE(ld_s >= n && ld_s % 4 == 0, HC_ESHAPE, "%s: ld_s=%lld must be >= n and a multiple of 4",
               fn, (long long)ld_s);
    HC_REQUIRE(ld_z >= 4 * nb && ld_z % 4 == 0, HC_ESHAPE,
               "%s: ld_z=%lld must be >= 4*ceil(k/3)=%lld and a multiple of 4", fn, (long long)ld_z,
               (long long)(4 * nb));
    if (m == 0) return HC_OK;
    HC_REQUIRE(E && S && Z, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned4(E) && aligned16(S) && aligned16(Z), HC_EALIGN,
               "%s: S and Z need 16-byte alignment, E 4-byte", fn);
    return launch_encode(E, k, n, S, m, ld_s, Z, ld_z, as_stream(stream));
}

hc_status hc_shade_spectral(const hc_paths* paths, const hc_spectral_assets* A, const float* T,
                            float* xyz, void* stream) {
    clear_error();
    const char* fn = "hc_shade_spectral";
    hc_status s = check_paths_struct(paths, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(A != nullptr, HC_EINVAL, "%s: assets is NULL", fn);
    HC_REQUIRE(A->n >= 1 && A->n <= kMaxN, HC_ESHAPE, "%s: n=%d outside [1, %d]", fn, A->n, kMaxN);
    HC_REQUIRE(A->ld >= A->n && A->ld % 4 == 0 && A->ld_illum >= A->n && A->ld_illum % 4 == 0,
               HC_ESHAPE, "%s: ld/ld_illum must be >= n and multiples of 4", fn);
    HC_REQUIRE(A->ld < (int64_t(1) << 30), HC_ESHAPE, "%s: ld must be < 2^30", fn);
    HC_REQUIRE(A->n_texels >= 1 && A->n_texels < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_texels outside [1, 2^32)", fn);
    HC_REQUIRE(A->n_illum >= 1 && A->n_illum <= (1 << 24), HC_ESHAPE, "%s: n_illum outside [1, 2^24]",
               fn);
    if (paths->n_pixels == 0) return HC_OK;
    HC_REQUIRE(A->refl && A->illum && T && xyz, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned16(A->refl) && aligned16(A->illum), HC_EALIGN,
               "%s: refl/illum need 16-byte alignment", fn);
    HC_REQUIRE(aligned4(T) && aligned4(xyz), HC_EALIGN, "%s: T/xyz need 4-byte alignment", fn);
    return launch_shade_spectral(*paths, *A, T, xyz, as_stream(stream));
}

hc_status hc_shade_latent(const hc_paths* paths, const hc_latent_assets* A, int32_t block_first,
                          int32_t block_count, float* zimg, int64_t ld_zimg, void* stream) {
    clear_error();
    const char* fn = "hc_shade_latent";
    hc_status s = check_paths_struct(paths, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(A != nullptr, HC_EINVAL, "%s: assets is NULL", fn);
    HC_REQUIRE(A->k >= 1 && A->k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, A->k, kMaxK);
    const int nb = int(ceil_div(A->k, 3));
    HC_REQUIRE(block_first >= 0 && block_count >= 1 && block_first + block_count <= nb, HC_ESHAPE,
               "%s: blocks [%d, %d) outside the code's %d blocks", fn, block_first,
               block_first + block_count, nb);
    HC_REQUIRE(A->ld >= 4 * nb && A->ld % 4 == 0 && A->ld_illum >= 4 * nb && A->ld_illum % 4 == 0,
               HC_ESHAPE, "%s: ld/ld_illum must be >= 4*ceil(k/3) and multiples of 4", fn);
    HC_REQUIRE(A->ld < (int64_t(1) << 31), HC_ESHAPE, "%s: ld must be < 2^31", fn);
    HC_REQUIRE(ld_zimg >= 4 * nb && ld_zimg % 4 == 0, HC_ESHAPE,
               "%s: ld_zimg must be >= 4*ceil(k/3) and a multiple of 4", fn);
    HC_REQUIRE(A->n_texels >= 1 && A->n_texels < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_texels outside [1, 2^32)", fn);
    HC_REQUIRE(A->n_illum >= 1 && A->n_illum <= (1 << 24), HC_ESHAPE, "%s: n_illum outside [1, 2^24]",
               fn);
    if (paths->n_pixels == 0) return HC_OK;
    HC_REQUIRE(A->codes && A->illum_codes && zimg, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned16(A->codes) && aligned16(A->illum_codes) && aligned16(zimg), HC_EALIGN,
               "%s: codes/illum_codes/zimg need 16-byte alignment", fn);
    return launch_shade_latent(*paths, *A, block_first, block_count, zimg, ld_zimg,
                               as_stream(stream));
}

hc_status hc_shade_latent_xyz(const hc_paths* paths, const hc_latent_assets* A, const float* M, float* xyz,
                              void* stream) {
    clear_error();
    const char* fn = "hc_shade_latent_xyz";
    hc_status s = check_paths_struct(paths, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(A != nullptr, HC_EINVAL, "%s: assets is NULL", fn);
    HC_REQUIRE(A->k >= 1 && A->k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, A->k, kMaxK);
    const int nb = int(ceil_div(A->k, 3));
    HC_REQUIRE(A->ld >= 4 * nb && A->ld % 4 == 0 && A->ld_illum >= 4 * nb && A->ld_illum % 4 == 0,
               HC_ESHAPE, "%s: ld/ld_illum must be >= 4*ceil(k/3) and multiples of 4", fn);
    HC_REQUIRE(A->ld < (int64_t(1) << 31), HC_ESHAPE, "%s: ld must be < 2^31", fn);
    HC_REQUIRE(A->n_texels >= 1 && A->n_texels < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_texels outside [1, 2^32)", fn);
    HC_REQUIRE(A->n_illum >= 1 && A->n_illum <= (1 << 24), HC_ESHAPE, "%s: n_illum outside [1, 2^24]",
               fn);
    if (paths->n_pixels == 0) return HC_OK;
    HC_REQUIRE(A->codes && A->illum_codes && M && xyz, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned16(A->codes) && aligned16(A->illum_codes), HC_EALIGN,
               "%s: codes/illum_codes need 16-byte alignment", fn);
    HC_REQUIRE(aligned4(M) && aligned4(xyz), HC_EALIGN, "%s: M/xyz need 4-byte alignment", fn);
    return launch_shade_latent_xyz(*paths, *A, M, xyz, as_stream(stream));
}

hc_status hc_decode_matrix(const float* D, int32_t n, int32_t k, const float* T, float* M, void* stream) {
    clear_error();
    const char* fn = "hc_decode_matrix";
    HC_REQUIRE(k >= 1 && k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, k, kMaxK);
    HC_REQUIRE(n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: n=%d outside [1, %d]", fn, n, kMaxN);
    HC_REQUIRE(D && T && M, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned4(D) && aligned4(T) && aligned4(M), HC_EALIGN, "%s: D/T/M need 4-byte alignment",
               fn);
    return launch_decode_matrix(D, n, k, T, M, as_stream(stream));
}

hc_status hc_decode_xyz(const float* D, int32_t n, int32_t k, const float* T, const float* zimg,
                        int64_t n_pixels, int64_t ld_zimg, float* xyz, float* spectra,
                        int64_t ld_spectra, void* stream) {
    clear_error();
    const char* fn = "hc_decode_xyz";
    HC_REQUIRE(k >= 1 && k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, k, kMaxK);
    HC_REQUIRE(n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: n=%d outside [1, %d]", fn, n, kMaxN);
    HC_REQUIRE(n_pixels >= 0 && n_pixels < (int64_t(1) << 34), HC_ESHAPE, "%s: bad n_pixels", fn);
    const int64_t nb = ceil_div(k, 3);
    HC_REQUIRE(ld_zimg >= 4 * nb && ld_zimg % 4 == 0, HC_ESHAPE,
               "%s: ld_zimg must be >= 4*ceil(k/3) and a multiple of 4", fn);
    if (spectra) HC_REQUIRE(ld_spectra >= n, HC_ESHAPE, "%s: ld_spectra < n", fn);
    if (n_pixels == 0) return HC_OK;
    HC_REQUIRE(D && T && zimg && xyz, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned16(zimg) && aligned4(D) && aligned4(T) && aligned4(xyz) &&
                   (!spectra || aligned4(spectra)),
               HC_EALIGN, "%s: zimg needs 16-byte alignment, the rest 4-byte", fn);
    return launch_decode(D, n, k, T, zimg, n_pixels, ld_zimg, xyz, spectra, ld_spectra,
                         as_stream(stream));
}

static hc_status check_tables(const void* frames, int32_t n_frames, const void* tiles,
                              const int32_t* n_tiles, int32_t max_tiles, int32_t grid, const char* fn) {
    HC_REQUIRE(frames && tiles && n_tiles, HC_EINVAL, "%s: NULL table pointer", fn);
    HC_REQUIRE(aligned8(frames) && aligned8(tiles) && aligned4(n_tiles), HC_EALIGN,
               "%s: tables must be 8-byte aligned", fn);
    HC_REQUIRE(n_frames >= 1 && max_tiles >= 1, HC_ESHAPE, "%s: n_frames and max_tiles must be >= 1",
               fn);
    HC_REQUIRE(grid <= 65536, HC_ESHAPE, "%s: grid must be <= 65536 (<= 0: chosen by the library)", fn);
    return HC_OK;
}

hc_status hc_shade_latent_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                                const int32_t* n_tiles, int32_t max_tiles, int32_t k, int32_t grid,
                                void* stream) {
    clear_error();
    const char* fn = "hc_shade_latent_tiles";
    hc_status s = check_tables(frames, n_frames, tiles, n_tiles, max_tiles, grid, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(k >= 1 && k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, k, kMaxK);
    return launch_shade_latent_tiles(frames, n_frames, tiles, n_tiles, max_tiles, k, grid,
                                     as_stream(stream));
}

hc_status hc_shade_latent_xyz_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                                    const int32_t* n_tiles, int32_t max_tiles, int32_t k, const float* M,
                                    int32_t grid, void* stream) {
    clear_error();
    const char* fn = "hc_shade_latent_xyz_tiles";
    hc_status s = check_tables(frames, n_frames, tiles, n_tiles, max_tiles, grid, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(k >= 1 && k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, k, kMaxK);
    HC_REQUIRE(M && aligned4(M), HC_EINVAL, "%s: M NULL or misaligned", fn);
    return launch_shade_latent_xyz_tiles(frames, n_frames, tiles, n_tiles, max_tiles, k, M, grid,
                                         as_stream(stream));
}

hc_status hc_shade_spectral_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                                  const int32_t* n_tiles, int32_t max_tiles, int32_t n, const float* T,
                                  int32_t grid, void* stream) {
    clear_error();
    const char* fn = "hc_shade_spectral_tiles";
    hc_status s = check_tables(frames, n_frames, tiles, n_tiles, max_tiles, grid, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: n=%d outside [1, %d]", fn, n, kMaxN);
    HC_REQUIRE(T && aligned4(T), HC_EINVAL, "%s: T NULL or misaligned", fn);
    return launch_shade_spectral_tiles(frames, n_frames, tiles, n_tiles, max_tiles, n, T, grid,
                                       as_stream(stream));
}

hc_status hc_decode_tiles(const hc_frame* frames, int32_t n_frames, const hc_tile* tiles,
                          const int32_t* n_tiles, int32_t max_tiles, const float* D, int32_t n,
                          int32_t k, const float* T, int32_t grid, void* stream) {
    clear_error();
    const char* fn = "hc_decode_tiles";
    hc_status s = check_tables(frames, n_frames, tiles, n_tiles, max_tiles, grid, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(k >= 1 && k <= kMaxK && n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: bad k or n", fn);
    HC_REQUIRE(D && T && aligned4(D) && aligned4(T), HC_EINVAL, "%s: D/T NULL or misaligned", fn);
    return launch_decode_tiles(frames, n_frames, tiles, n_tiles, max_tiles, D, n, k, T, grid,
                               as_stream(stream));
}

hc_status hc_encode_jobs(const hc_encode_job* jobs, const int32_t* n_jobs, int32_t max_jobs,
                         const float* E, int32_t k, int32_t n, int32_t grid, void* stream) {
    clear_error();
    const char* fn = "hc_encode_jobs";
    HC_REQUIRE(jobs && n_jobs && E, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned8(jobs) && aligned4(n_jobs) && aligned4(E), HC_EALIGN, "%s: misaligned table",
               fn);
    HC_REQUIRE(k >= 1 && k <= kMaxK && n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: bad k or n", fn);
    HC_REQUIRE(max_jobs >= 1 && grid <= 65536, HC_ESHAPE, "%s: bad max_jobs or grid", fn);
    return launch_encode_jobs(jobs, n_jobs, max_jobs, E, k, n, grid, as_stream(stream));
}

hc_status hc_check_paths(const hc_paths* paths, int64_t n_texels, int32_t n_illum, uint64_t* counts,
                         void* stream) {
    clear_error();
    const char* fn = "hc_check_paths";
    hc_status s = check_paths_struct(paths, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(counts != nullptr && aligned8(counts), HC_EINVAL, "%s: counts NULL or misaligned", fn);
    HC_REQUIRE(n_texels >= 0 && n_illum >= 0, HC_ESHAPE, "%s: negative asset sizes", fn);
    return launch_check_paths(*paths, n_texels, n_illum, counts, as_stream(stream));
}

size_t hc_codec_workspace_size(int32_t k, int32_t n, int64_t N) {
    if (k < 1 || k > kMaxK || n < 1 || n > kMaxN || N < 1) return 0;
    return codec_workspace_size(k, n, N);
}

namespace {

// Every check of hc_codec_step except the workspace's.
hc_status check_codec_args(const hc_codec_args* a, const char* fn) {
    HC_REQUIRE(a != nullptr, HC_EINVAL, "%s: args is NULL", fn);
    HC_REQUIRE(a->k >= 1 && a->k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, a->k, kMaxK);
    HC_REQUIRE(a->n >= 1 && a->n <= kMaxN, HC_ESHAPE, "%s: n=%d outside [1, %d]", fn, a->n, kMaxN);
    HC_REQUIRE(a->dtype == 0 || a->dtype == 1, HC_EINVAL, "%s: dtype must be 0 or 1", fn);
    HC_REQUIRE(a->objective == HC_CODEC_L2 || a->objective == HC_CODEC_EQ8, HC_EINVAL,
               "%s: objective must be HC_CODEC_L2 or HC_CODEC_EQ8", fn);
    if (a->objective == HC_CODEC_EQ8) {
        HC_REQUIRE(a->T != nullptr, HC_EINVAL, "%s: HC_CODEC_EQ8 needs T", fn);
        const double w[4] = {a->w_e2e, a->w_rec, a->w_code, a->w_col};
        for (double x : w)
            HC_REQUIRE(x >= 0 && x < HUGE_VAL, HC_EINVAL, "%s: Eq. 8 weights must be finite and >= 0", fn);
        HC_REQUIRE(a->cos_eps > 0 && a->cos_eps < HUGE_VAL, HC_EINVAL, "%s: cos_eps must be > 0", fn);
    }
    HC_REQUIRE(a->N >= 1 && a->N < (int64_t(1) << 31), HC_ESHAPE, "%s: N outside [1, 2^31)", fn);
    HC_REQUIRE(a->beta > 0, HC_EINVAL, "%s: beta must be > 0", fn);
    HC_REQUIRE(a->ld_a >= a->n && a->ld_b >= a->n, HC_ESHAPE, "%s: ld_a/ld_b < n", fn);
    HC_REQUIRE(a->Wt_E && a->Wt_D && a->A && a->B && a->loss, HC_EINVAL, "%s: NULL pointer", fn);
    if (a->draw) {
        HC_REQUIRE(!a->idx_a && !a->idx_b, HC_EINVAL, "%s: draw excludes idx_a / idx_b", fn);
        HC_REQUIRE(a->rows_a >= 1 && a->rows_a < (int64_t(1) << 32) && a->rows_b >= 1 &&
                       a->rows_b < (int64_t(1) << 32),
                   HC_ESHAPE, "%s: drawn rows need rows_a, rows_b in [1, 2^32)", fn);
        HC_REQUIRE(!a->draw->ctr_scale_dev || aligned8(a->draw->ctr_scale_dev), HC_EALIGN,
                   "%s: draw counter misaligned", fn);
    } else {
        if (a->idx_a) HC_REQUIRE(a->rows_a >= 1, HC_ESHAPE, "%s: rows_a must be >= 1 with idx_a", fn);
        if (a->idx_b) HC_REQUIRE(a->rows_b >= 1, HC_ESHAPE, "%s: rows_b must be >= 1 with idx_b", fn);
        if (!a->idx_a) HC_REQUIRE(a->rows_a >= a->N, HC_ESHAPE, "%s: rows_a < N without idx_a", fn);
        if (!a->idx_b) HC_REQUIRE(a->rows_b >= a->N, HC_ESHAPE, "%s: rows_b < N without idx_b", fn);
    }
    const size_t esz = a->dtype ? 8 : 4;
    auto al = [&](const void* p) { return (reinterpret_cast<uintptr_t>(p) % esz) == 0; };
    HC_REQUIRE(al(a->Wt_E) && al(a->Wt_D) && al(a->A) && al(a->B) && al(a->loss) &&
                   (!a->grad_E || al(a->grad_E)) && (!a->grad_D || al(a->grad_D)) &&
                   (a->objective != HC_CODEC_EQ8 || al(a->T)),
               HC_EALIGN, "%s: arrays must be aligned to their element size", fn);
    if (a->adam) {
        const hc_adam* m = a->adam;
        HC_REQUIRE(m->m_E && m->v_E && m->m_D && m->v_D && m->step, HC_EINVAL,
                   "%s: adam state has a NULL pointer", fn);
        HC_REQUIRE(al(m->m_E) && al(m->v_E) && al(m->m_D) && al(m->v_D) && aligned8(m->step),
                   HC_EALIGN, "%s: adam state misaligned", fn);
        HC_REQUIRE(m->lr > 0 && m->beta1 >= 0 && m->beta1 < 1 && m->beta2 >= 0 && m->beta2 < 1 &&
                       m->eps > 0,
                   HC_EINVAL, "%s: adam hyper-parameters out of range", fn);
    }
    return HC_OK;
}

}  // namespace

hc_status hc_codec_step(const hc_codec_args* a) {
    clear_error();
    const char* fn = "hc_codec_step";
    const hc_status s = check_codec_args(a, fn);
    if (s != HC_OK) return s;
    const size_t need = codec_workspace_size(a->k, a->n, a->N);
    HC_REQUIRE(a->workspace != nullptr && a->workspace_bytes >= need && aligned8(a->workspace),
               HC_ENOMEM, "%s: workspace needs %zu bytes (8-byte aligned), got %zu", fn, need,
               a->workspace_bytes);
    return launch_codec_step(*a);
}

hc_status hc_codec_step_static(const hc_codec_args* a) {
    clear_error();
    const char* fn = "hc_codec_step_static";
    const hc_status s = check_codec_args(a, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(a->workspace == nullptr && a->workspace_bytes == 0, HC_EINVAL,
               "%s: takes no workspace (workspace must be NULL and workspace_bytes 0)", fn);
    const size_t need = codec_static_need(*a);
    HC_REQUIRE(need <= size_t(HC_CODEC_STATIC_SCRATCH_BYTES), HC_ENOMEM,
               "%s: this shape needs %zu bytes of scratch, above the %zu of the static array", fn, need,
               size_t(HC_CODEC_STATIC_SCRATCH_BYTES));
    return launch_codec_step_static(*a);
}

hc_status hc_upsample(const hc_mlp* net, int32_t precision, const float* rgb, int64_t m,
                      int64_t ld_rgb, float* Z, int64_t ld_z, void* stream) {
    clear_error();
    const char* fn = "hc_upsample";
    HC_REQUIRE(net != nullptr, HC_EINVAL, "%s: net is NULL", fn);
    HC_REQUIRE(net->hidden == 128, HC_EUNSUPPORTED, "%s: hidden width %d (only 128 is compiled)", fn,
               net->hidden);
    HC_REQUIRE(net->k >= 1 && net->k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, net->k, kMaxK);
    HC_REQUIRE(precision == HC_MLP_F32 || precision == HC_MLP_F16, HC_EINVAL,
               "%s: precision must be HC_MLP_F32 or HC_MLP_F16", fn);
    HC_REQUIRE(m >= 0 && m < (int64_t(1) << 40), HC_ESHAPE, "%s: m=%lld out of range", fn, (long long)m);
    HC_REQUIRE(ld_rgb >= 3, HC_ESHAPE, "%s: ld_rgb < 3", fn);
    HC_REQUIRE(ld_z >= 4 * ceil_div(net->k, 3), HC_ESHAPE, "%s: ld_z < 4 ceil(k/3)", fn);
    if (m == 0) return HC_OK;
    HC_REQUIRE(net->W1 && net->b1 && net->W2 && net->b2 && net->W3 && net->b3 && rgb && Z, HC_EINVAL,
               "%s: NULL pointer", fn);
    HC_REQUIRE(aligned4(net->W1) && aligned4(net->b1) && aligned4(net->W2) && aligned4(net->b2) &&
                   aligned4(net->W3) && aligned4(net->b3) && aligned4(rgb) && aligned4(Z),
               HC_EALIGN, "%s: arrays must be 4-byte aligned", fn);
    return launch_upsample(*net, precision, rgb, m, ld_rgb, Z, ld_z, as_stream(stream));
}

int64_t hc_upsample_param_count(int32_t k, int32_t hidden) {
    if (k < 1 || k > kMaxK || hidden != 128) return -1;
    return upsample_param_count(k);
}

size_t hc_upsample_train_workspace_size(int32_t k, int64_t N) {
    if (k < 1 || k > kMaxK || N < 1) return 0;
    return upsample_train_workspace_size(k, N);
}

hc_status hc_upsample_train_step(const hc_upsample_train_args* a) {
    clear_error();
    const char* fn = "hc_upsample_train_step";
    HC_REQUIRE(a != nullptr, HC_EINVAL, "%s: args is NULL", fn);
    HC_REQUIRE(a->hidden == 128, HC_EUNSUPPORTED, "%s: hidden width %d (only 128 is compiled)", fn,
               a->hidden);
    HC_REQUIRE(a->k >= 1 && a->k <= kMaxK, HC_ESHAPE, "%s: k=%d outside [1, %d]", fn, a->k, kMaxK);
    HC_REQUIRE(a->N >= 1 && a->N < (int64_t(1) << 31), HC_ESHAPE, "%s: N outside [1, 2^31)", fn);
    HC_REQUIRE(a->ld_rgb >= 3 && a->ld_z >= 4 * ceil_div(a->k, 3), HC_ESHAPE, "%s: row stride too small",
               fn);
    HC_REQUIRE(a->params && a->rgb && a->z_gt && a->M && a->loss, HC_EINVAL, "%s: NULL pointer", fn);
    if (a->draw) {
        HC_REQUIRE(!a->idx, HC_EINVAL, "%s: draw excludes idx", fn);
        HC_REQUIRE(a->rows >= 1 && a->rows < (int64_t(1) << 32), HC_ESHAPE,
                   "%s: drawn rows need rows in [1, 2^32)", fn);
        HC_REQUIRE(!a->draw->ctr_scale_dev || aligned8(a->draw->ctr_scale_dev), HC_EALIGN,
                   "%s: draw counter misaligned", fn);
    } else if (a->idx) {
        HC_REQUIRE(a->rows >= 1, HC_ESHAPE, "%s: rows must be >= 1 with idx", fn);
    } else {
        HC_REQUIRE(a->rows >= a->N, HC_ESHAPE, "%s: rows < N without idx", fn);
    }
    for (double w : a->white)
        HC_REQUIRE(w > 0 && w < HUGE_VAL, HC_EINVAL, "%s: the white must be positive and finite", fn);
    HC_REQUIRE(a->w_max >= 0 && a->w_max < HUGE_VAL && a->w_col >= 0 && a->w_col < HUGE_VAL, HC_EINVAL,
               "%s: loss weights must be finite and >= 0", fn);
    HC_REQUIRE(aligned4(a->params) && aligned4(a->rgb) && aligned4(a->z_gt) && aligned4(a->M) &&
                   aligned4(a->loss) && (!a->grad || aligned4(a->grad)),
               HC_EALIGN, "%s: arrays must be 4-byte aligned", fn);
    if (a->opt) {
        const hc_adamw* o = a->opt;
        HC_REQUIRE(o->m && o->v && o->step, HC_EINVAL, "%s: optimizer state has a NULL pointer", fn);
        HC_REQUIRE(aligned4(o->m) && aligned4(o->v) && aligned8(o->step), HC_EALIGN,
                   "%s: optimizer state misaligned", fn);
        HC_REQUIRE(o->lr > 0 && o->beta1 >= 0 && o->beta1 < 1 && o->beta2 >= 0 && o->beta2 < 1 &&
                       o->eps > 0 && o->weight_decay >= 0 && o->max_grad_norm > 0,
                   HC_EINVAL, "%s: optimizer hyper-parameters out of range", fn);
    }
    const size_t need = upsample_train_workspace_size(a->k, a->N);
    HC_REQUIRE(a->workspace != nullptr && a->workspace_bytes >= need &&
                   (reinterpret_cast<uintptr_t>(a->workspace) & 255u) == 0,
               HC_ENOMEM, "%s: workspace needs %zu bytes (256-byte aligned), got %zu", fn, need,
               a->workspace_bytes);
    return launch_upsample_train(*a);
}

hc_status hc_codec_weights(const void* Wt_E, const void* Wt_D, int32_t k, int32_t n, int32_t dtype,
                           double beta, float* E, float* D, void* stream) {
    clear_error();
    const char* fn = "hc_codec_weights";
    HC_REQUIRE(k >= 1 && k <= kMaxK && n >= 1 && n <= kMaxN, HC_ESHAPE, "%s: bad k or n", fn);
    HC_REQUIRE(dtype == 0 || dtype == 1, HC_EINVAL, "%s: dtype must be 0 or 1", fn);
    HC_REQUIRE(beta > 0, HC_EINVAL, "%s: beta must be > 0", fn);
    HC_REQUIRE(Wt_E && Wt_D && E && D, HC_EINVAL, "%s: NULL pointer", fn);
    return launch_codec_weights(Wt_E, Wt_D, k, n, dtype, beta, E, D, as_stream(stream));
}

size_t hc_gen_workspace_size(int64_t n_pixels) {
    return n_pixels < 0 ? 0 : gen_workspace_size(n_pixels);
}

static hc_status check_gen(const hc_path_gen* g, const char* fn) {
    HC_REQUIRE(g != nullptr, HC_EINVAL, "%s: spec is NULL", fn);
    HC_REQUIRE(g->n_pixels >= 0 && g->spp >= 1, HC_ESHAPE, "%s: bad n_pixels/spp", fn);
    HC_REQUIRE(g->n_pixels <= (int64_t(1) << 40) / g->spp, HC_ESHAPE, "%s: too many paths", fn);
    HC_REQUIRE(0 <= g->l_min && g->l_min <= g->l_max && g->l_max <= 255, HC_ESHAPE,
               "%s: need 0 <= l_min <= l_max <= 255", fn);
    HC_REQUIRE(g->n_illum >= 1 && g->n_illum <= (1 << 24), HC_ESHAPE, "%s: n_illum outside [1, 2^24]",
               fn);
    HC_REQUIRE(g->n_tex >= 1 && g->n_tex < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_tex outside [1, 2^32)", fn);
    return HC_OK;
}

hc_status hc_gen_path_headers(const hc_path_gen* g, uint32_t* hdr, uint32_t* pix_first,
                              uint64_t* n_vertices, void* workspace, size_t workspace_bytes,
                              void* stream) {
    clear_error();
    const char* fn = "hc_gen_path_headers";
    hc_status s = check_gen(g, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(n_vertices && aligned8(n_vertices), HC_EINVAL, "%s: n_vertices NULL/misaligned", fn);
    if (g->n_pixels > 0) {
        HC_REQUIRE(hdr && pix_first && aligned4(hdr) && aligned4(pix_first), HC_EINVAL,
                   "%s: hdr/pix_first NULL or misaligned", fn);
    }
    const size_t need = gen_workspace_size(g->n_pixels);
    HC_REQUIRE(workspace_bytes >= need && (need == 0 || (workspace && aligned8(workspace))), HC_ENOMEM,
               "%s: workspace needs %zu bytes, got %zu", fn, need, workspace_bytes);
    return launch_gen_headers(*g, hdr, pix_first, n_vertices, workspace, workspace_bytes,
                              as_stream(stream));
}

hc_status hc_gen_path_vertices(const hc_path_gen* g, const uint32_t* pix_first, uint32_t* vtx,
                               int64_t n_vertices, void* stream) {
    clear_error();
    const char* fn = "hc_gen_path_vertices";
    hc_status s = check_gen(g, fn);
    if (s != HC_OK) return s;
    HC_REQUIRE(n_vertices >= 0 && n_vertices < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_vertices outside [0, 2^32)", fn);
    if (g->n_pixels == 0) return HC_OK;
    HC_REQUIRE(pix_first && aligned4(pix_first), HC_EINVAL, "%s: pix_first NULL/misaligned", fn);
    HC_REQUIRE(n_vertices == 0 || (vtx && aligned8(vtx)), HC_EINVAL, "%s: vtx NULL/misaligned", fn);
    return launch_gen_vertices(*g, pix_first, vtx, n_vertices, as_stream(stream));
}

hc_status hc_gen_indices(uint64_t seed, uint64_t ctr0, const int64_t* ctr_scale_dev, int64_t count,
                         int64_t n, uint32_t* out, void* stream) {
    clear_error();
    const char* fn = "hc_gen_indices";
    HC_REQUIRE(count >= 0 && count < (int64_t(1) << 40), HC_ESHAPE, "%s: bad count", fn);
    HC_REQUIRE(n >= 1 && n < (int64_t(1) << 32), HC_ESHAPE, "%s: n outside [1, 2^32)", fn);
    if (count == 0) return HC_OK;
    HC_REQUIRE(out && aligned4(out), HC_EINVAL, "%s: out NULL/misaligned", fn);
    HC_REQUIRE(!ctr_scale_dev || aligned8(ctr_scale_dev), HC_EALIGN, "%s: counter misaligned", fn);
    return launch_gen_indices(seed, ctr0, ctr_scale_dev, count, n, out, as_stream(stream));
}

hc_status hc_gather_probe(const uint32_t* vtx, int64_t n_vertices, const float* table, int64_t n_rows,
                          int64_t ld, int32_t row_floats, int32_t unroll, int32_t lanes_per_row,
                          int32_t grid, float* out, void* stream) {
    clear_error();
    const char* fn = "hc_gather_probe";
    HC_REQUIRE(n_vertices >= 0 && n_vertices < (int64_t(1) << 32), HC_ESHAPE,
               "%s: n_vertices outside [0, 2^32)", fn);
    HC_REQUIRE(n_rows >= 1 && n_rows < (int64_t(1) << 32), HC_ESHAPE, "%s: n_rows outside [1, 2^32)", fn);
    HC_REQUIRE(unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8, HC_EINVAL,
               "%s: unroll must be 1, 2, 4 or 8 (got %d)", fn, unroll);
    HC_REQUIRE(lanes_per_row == 1 || lanes_per_row == 8, HC_EINVAL, "%s: lanes_per_row must be 1 or 8", fn);
    HC_REQUIRE(row_floats >= 1 && row_floats <= (lanes_per_row == 1 ? 16 : 128), HC_ESHAPE,
               "%s: row_floats=%d outside [1, %d] for %d lane(s) per row", fn, row_floats,
               lanes_per_row == 1 ? 16 : 128, lanes_per_row);
    HC_REQUIRE(ld >= row_floats && ld % 4 == 0 && ld < (int64_t(1) << 31), HC_ESHAPE,
               "%s: ld must be >= row_floats, a multiple of 4 and < 2^31", fn);
    HC_REQUIRE(grid >= 1 && grid <= (1 << 20), HC_ESHAPE, "%s: grid outside [1, 2^20]", fn);
    HC_REQUIRE(table && out && (vtx || n_vertices == 0), HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned16(table) && aligned4(out) && aligned8(vtx), HC_EALIGN,
               "%s: table/vtx/out need 16/8/4-byte alignment", fn);
    return launch_gather_probe(reinterpret_cast<const uint2*>(vtx), uint32_t(n_vertices), table,
                               uint32_t(n_rows), uint32_t(ld), row_floats, unroll, lanes_per_row, out,
                               grid, as_stream(stream));
}

hc_status hc_stream_probe(const float* src, float* dst, int64_t n16, int32_t mode, int32_t grid, void* stream) {
    clear_error();
    const char* fn = "hc_stream_probe";
    HC_REQUIRE(mode == 0 || mode == 1, HC_EINVAL, "%s: mode must be 0 (read) or 1 (copy), got %d", fn, mode);
    HC_REQUIRE(n16 >= 0 && n16 < (int64_t(1) << 40), HC_ESHAPE, "%s: n16 outside [0, 2^40)", fn);
    HC_REQUIRE(grid >= 1 && grid <= (1 << 20), HC_ESHAPE, "%s: grid outside [1, 2^20]", fn);
    HC_REQUIRE(dst && (src || n16 == 0), HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned16(src) && (mode == 0 ? aligned4(dst) : aligned16(dst)), HC_EALIGN,
               "%s: src needs 16-byte alignment, dst 4 (read) or 16 (copy)", fn);
    if (mode == 1 && n16 == 0) return HC_OK;
    return launch_stream_probe(src, dst, uint64_t(n16), mode, grid, as_stream(stream));
}

hc_status hc_alu_probe(int32_t op, float* out, int32_t grid, void* stream) {
    clear_error();
    const char* fn = "hc_alu_probe";
    HC_REQUIRE(op >= 0 && op <= 5, HC_EINVAL, "%s: op must be in [0, 5], got %d", fn, op);
    HC_REQUIRE(grid >= 1 && grid <= (1 << 20), HC_ESHAPE, "%s: grid outside [1, 2^20]", fn);
    HC_REQUIRE(out != nullptr, HC_EINVAL, "%s: NULL pointer", fn);
    HC_REQUIRE(aligned4(out), HC_EALIGN, "%s: out needs 4-byte alignment", fn);
    return hc::launch_alu_probe(op, out, grid, as_stream(stream));
}

}  // extern "C"
