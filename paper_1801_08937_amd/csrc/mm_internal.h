// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mapmaker.h"

namespace mm {

// An error carried from deep inside a call up to the C-ABI boundary, where it
// becomes the call's status and the context's last-error message.
struct Error : std::runtime_error {
    mm_status code;
    Error(mm_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define MM_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::mm::Error(e_ == hipErrorOutOfMemory ? MM_E_OOM : MM_E_DEVICE,      \
                              std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define MM_CHECK(cond, code, msg)                                                      \
    do {                                                                               \
        if (!(cond)) throw ::mm::Error((code), (msg));                                 \
    } while (0)

// Owning device buffer.
struct DBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    // Grow-only.  Growing a buffer that queued kernels may still use waits
    // for the device first.
    void alloc(size_t b) {
        if (b <= bytes && ptr) return;
        if (ptr) (void)hipDeviceSynchronize();
        release();
        if (b == 0) return;
        hipError_t e = hipMalloc(&ptr, b);
        if (e != hipSuccess) {
            ptr = nullptr;
            throw Error(MM_E_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
        bytes = b;
    }
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// Per-stage timing with HIP events on the context's stream.
struct Profiler {
    bool on = false;
    struct Stage { double ms = 0; int64_t calls = 0; };
    std::map<std::string, Stage> stages;
    struct Pending { std::string name; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    void flush();  // synchronises on the recorded events
    ~Profiler();
};

struct Scope {
    Profiler *pr;
    hipStream_t s;
    const char *name;
    hipEvent_t a{}, b{};
    Scope(Profiler &p, hipStream_t st, const char *n);
    ~Scope();
};

}  // namespace mm

struct mm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string last_error;
    mm::Profiler prof;
    // reusable workspace
    mm::DBuf tod_a, tod_b;         // TOD temporaries for A applies
    mm::DBuf red;                  // reduction partials
    mm::DBuf scal;                 // small device scalars
    mm::DBuf gram_part, coef_g;    // MFMA Gram partials, coarse right-hand sides
    mm::DBuf xpack;                // map repacked for P: (I, Q, U, 0) records, or I and (Q, U) split
    mm::DBuf pt_part;              // per-segment partial maps of the sliced P^T
    mm::DBuf tod_c;                // template filter: filtered TOD, ground sums and amplitudes
    // Bumped whenever one of the workspaces above is reallocated: captured
    // graphs hold their addresses and are re-captured when it changes.
    uint64_t ws_gen = 0;
    hipStream_t cap = nullptr;     // private stream for graph capture
    double *pinned = nullptr;      // host pinned scratch (scalar readback)
    size_t pinned_bytes = 0;
    int n_cu = 256;
};

namespace mm {
// Grow a context workspace, recording the reallocation.
inline void ws_alloc(mm_ctx *ctx, DBuf &b, size_t bytes) {
    if (b.ptr && bytes <= b.bytes) return;
    b.alloc(bytes);
    ++ctx->ws_gen;
}
}  // namespace mm

struct mm_pointing {
    int64_t n_samp = 0;
    int32_t n_pix_total = 0;
    int32_t n_obs = 0;
    int64_t n_valid = 0;
    mm_precision prec = MM_F64;
    // map components: IQU (3 per pixel), I (1: weights 1, no angles kept) or
    // QU (2: weights cos 2psi, sin 2psi)
    mm_stokes stokes = MM_STOKES_IQU;
    int32_t nc = 3;
    int64_t n() const { return (int64_t)nc * n_obs; }
    mm::DBuf hits, obs_pix, j, w, perm, ws, off;
    mm::DBuf psi;  // f64[n_samp] angles (FP64 form only)
    // Map copies of the single-column IQU P (with a grid): p_copies copies,
    // one per scan direction found, each ordered by first touch along its
    // samples.  p_slot[g n_obs + c] is pixel c's slot in copy g (counted over
    // all copies) and p_j[t] the slot of sample t's pixel in its chunk's copy
    // (-1 flagged), so the pixels a wave gathers along the scan share cache
    // lines.  Without a grid the slot is the compact id and there is one copy.
    mm::DBuf p_slot, p_j;
    int32_t p_copies = 0;
    mm::DBuf p_chunk_grp;  // int32 copy (scan direction) of each 4,096-sample chunk
    int32_t max_seg = 0;
    // Order in which P^T visits the compact pixels (empty = ascending).  Each
    // pixel's own sum is independent of it; it only shapes cache locality.
    mm::DBuf seg_order;
    int32_t grid_width = 0;
    int32_t p_blocks[7] = {0, 0, 0, 0, 0, 0, 0};  // tuned P grid per log2(nrhs); 0 = default
    // tuned: visit pixels in seg_order (1) or ascending (0) in the
    // one-wave-per-pixel P^T, per log2(nrhs); -1 = default (seg_order if set)
    int32_t pt_order[7] = {-1, -1, -1, -1, -1, -1, -1};
    // Sliced single-column P^T: observed pixels in slices of 64 (one pixel per
    // lane; neighbours on the map when a grid is set), the samples cut into
    // sl_S equal time segments.  Wave (s, g) walks its lanes' entries of
    // segment s in time order from sl_perm / sl_w, stored interleaved (entry k
    // of lane l at sl_base[s G + g] + 64 k + l, padding t = -1, w = 0).
    // With map copies (grid hint) the slices are cut per scan direction d:
    // lane pixels are virtual ids v = d n_obs + c in copy d's first-touch
    // order, each walking only its pixel's samples of direction d, so sl_G
    // counts sl_D direction blocks of slices and wave (s, g) writes partial
    // map s sl_D + g / (sl_G / sl_D).
    int32_t sl_G = 0, sl_S = 0, sl_D = 1;
    mm::DBuf sl_pix;   // int32[G * 64] compact pixel per lane, -1 past n_obs
    mm::DBuf sl_base;  // int64[G * S + 1] entry offsets, segment-major
    mm::DBuf sl_perm;  // int32 sample index per entry
    mm::DBuf sl_w;     // per entry: psi (FP64 form) or the weights (FP32 form)
};

struct mm_noise {
    int64_t n_samp = 0;
    int32_t n_int = 0, n_filters = 0, half_bw = 0;
    mm_noise_method method = MM_NOISE_DIRECT;
    mm_precision prec = MM_F64;
    std::vector<int64_t> h_istart;
    std::vector<int32_t> h_fid;
    std::vector<double> h_band;
    mm::DBuf istart, fid, band, band64;
    // direct band: per column count R = 2^li (li = 0..6), the number of
    // tiles in the intervals before each interval, int64[7][n_int + 1]
    // (device copy and host copy); built with the handle, read-only after
    mm::DBuf tile_pref;
    std::vector<int64_t> h_tile_pref;
    int32_t band_cl[7] = {0, 0, 0, 0, 0, 0, 0};  // tuned taps per LDS chunk per log2(nrhs); 0 = default
    bool band_small = false;  // one column in 512-sample tiles of 64 threads (short streams)
    // FFT: per-filter packed spectrum and block table
    int32_t fft_n = 0;       // real block length
    int32_t fft_valid = 0;   // valid outputs per block
    mm::DBuf fft_spec;       // per filter: A_k, B_k (2 * fft_n/2 doubles)
    mm::DBuf fft_tw;         // twiddles exp(-2 pi i m / (fft_n/2)), m < fft_n/2
    mm::DBuf fft_blocks;     // int64 pairs (first output sample, interval index)
    int64_t n_fft_blocks = 0;
    // polynomial template filter (method MM_NOISE_POLY): subscan table, the
    // weight of each subscan's interval, G_s^-1 per subscan ((p+1)^2 FP64,
    // zeros for a subscan fitted exactly) and the flag mask as bits
    int32_t pf_order = 0;
    int64_t pf_n_sub = 0;
    int64_t pf_max_len = 0;  // longest subscan (picks the apply's register cache)
    mm::DBuf pf_sub, pf_omega, pf_ginv, pf_mask;
    // ground templates (pf_nb bins, 0 = none): each sample's bin, 1 / sum of
    // w per bin, and the bin-sorted samples and weights interleaved per wave
    // (wave w = a chunk of a group of 64 bins: entries [gbase[w], gbase[w+1]),
    // lane = bin; gfirst[g] = first wave of group g)
    int32_t pf_nb = 0;
    int32_t pf_n_gwave = 0;
    mm::DBuf pf_gbin, pf_gwinv, pf_gbase, pf_gfirst, pf_gsp, pf_gsw;
};

struct mm_precond {
    int kind = 0;  // 0 = M_BD, 1 = M_2l
    int32_t n_obs = 0;
    int32_t nc = 3;  // map components per pixel (the pointing's)
    int64_t n() const { return (int64_t)nc * n_obs; }
    // f64[n_obs][nc (nc + 1) / 2] packed symmetric B_j^-1: (00, 01, 02, 11,
    // 12, 22) for IQU, (00, 01, 11) for QU, (00) for I; for M_BD also the
    // assembled blocks B_j themselves, packed the same way (M_BD^-1, used to
    // form A Z from the Arnoldi factorisation)
    mm::DBuf inv, blk;
    double rcond_min = 0;
    // M_2l
    int32_t k = 0;
    // Z, AZ: f64[k][n]; E: f64[k][k]; Einv: E^-1, column r at Einv[r k]
    mm::DBuf Z, AZ, E, Einv;
    // Arnoldi record
    int32_t arn_m = 0;
    mm::DBuf W;
    std::vector<double> H;  // (m+1) x m column-major
};

namespace mm {

// ---- launchers (defined in the .hip files) ----
// pointing.hip
void pointing_build_device(mm_ctx *ctx, mm_pointing *p, const int32_t *pix, const double *psi,
                           int32_t min_hits);
void pointing_set_grid_device(mm_ctx *ctx, mm_pointing *p, int32_t width, int32_t tile);
// (Re)build the sliced P^T layout; width > 0 groups 8 x 8 pixel blocks of a
// row-major grid of that width into slices, width 0 takes ascending pixels.
void pointing_slices_device(mm_ctx *ctx, mm_pointing *p, int32_t width);
// (Re)build the Morton map slots of the FP64 P (width > 0), or drop them.
void pointing_p_slots_device(mm_ctx *ctx, mm_pointing *p, int32_t width);

// tod_ops.hip
// The P, P^T and N^-1 launchers take an optional device scratch region of at
// least *_scratch_bytes(...) bytes (256-byte aligned); with nullptr they use
// (and grow) the context's workspaces instead.
size_t apply_P_scratch_bytes(const mm_pointing *p, int nrhs);
size_t apply_PT_scratch_bytes(const mm_pointing *p, int nrhs);
size_t noise_scratch_bytes(const mm_noise *nz, int nrhs);
void apply_P_dev(mm_ctx *ctx, const mm_pointing *p, int nrhs, const double *x, void *y,
                 char *scratch = nullptr);
void apply_PT_dev(mm_ctx *ctx, const mm_pointing *p, int nrhs, const void *z, double *x,
                  char *scratch = nullptr);
void noise_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z,
                     char *scratch = nullptr);
int band_tile_len(int nrhs, bool small);
void mask_tod_dev(mm_ctx *ctx, const mm_pointing *p, int nrhs, const void *tod_rm, void *y,
                  int *nonfinite_flag);
void pair_sum_diff_dev(mm_ctx *ctx, int64_t n, mm_precision prec, const void *a, const void *b,
                       void *plus, void *minus);
// FFT tables (spectra, twiddles, block table) for overlap-save blocks of
// n_fft real samples (16,384 or 32,768; 0 = pick by the measured time model)
void noise_fft_prepare(mm_ctx *ctx, mm_noise *nz, int n_fft);
// polyfilter.hip
int polyfilter_max_order();
void polyfilter_prepare(mm_ctx *ctx, const mm_pointing *p, mm_noise *nz,
                        const int32_t *ground_bin, int32_t n_ground_bins);
size_t polyfilter_scratch_bytes(const mm_noise *nz, int nrhs);
void polyfilter_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z,
                          char *scratch = nullptr);
bool noise_fft_supported(int half_bw, int64_t min_len);

// map_ops.hip
void mbd_build_dev(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, mm_precond *M,
                   int *n_bad);
void mbd_apply_dev(mm_ctx *ctx, const double *inv, int32_t n_obs, int nc, int nrhs,
                   const double *v, double *out, const double *dot_with, double *dot_partial,
                   int n_part);
inline int packed_sym(int nc) { return nc * (nc + 1) / 2; }

// Deterministic dot products of columns: out[r] = sum_i a[i R + r] b[i R + r]
// over n rows (two stages, fixed order).
void dot_cols(mm_ctx *ctx, int64_t n, int nrhs, const double *a, const double *b, double *out);
// Blocks of a two-stage column reduction over n_rows x nrhs elements.
int reduction_parts(int64_t n_rows, int nrhs = 1);

// Small dense helpers
void gram_mfma(mm_ctx *ctx, int64_t n, int ka, int kb, const double *X, int64_t x_rs,
               int64_t x_cs, const double *Y, int64_t y_rs, int64_t y_cs, double *C);
void gemv_t(mm_ctx *ctx, int64_t n, int ncol, const double *W, const double *v, double *h);
void gemv_n_sub(mm_ctx *ctx, int64_t n, int ncol, const double *W, const double *h, double *v);
void scale_copy(mm_ctx *ctx, int64_t n, const double *src, const double *s_dev, double *dst,
                int invert);
// U[c n + i] += g[c] r[i] (U column-major n x k; g on the device).
void rank1_add(mm_ctx *ctx, int64_t n, int k, const double *r, const double *g, double *U);
void matmul_small_right(mm_ctx *ctx, int64_t n, int kin, int kout, const double *V,
                        const double *Y, double *Zout);  // Zout = V Y, col-major
// Cholesky factor Lc of the k x k matrix E; E is symmetrised in place first.
void chol_small_dev(mm_ctx *ctx, int k, double *E, double *Lc, int *flag);
// E^-1 (column r at Einv[r k]) from the lower Cholesky factor Lc of E.
void coarse_inverse_dev(mm_ctx *ctx, int k, const double *Lc, double *Einv);
void m2l_apply_dev(mm_ctx *ctx, const mm_precond *M, int nrhs, const double *v, double *out,
                   double *dot_partial, int n_part);
void m2l_coef_dev(mm_ctx *ctx, const mm_precond *M, int nrhs, const double *v, double *c);

// PCG vector kernels on column-batched map vectors
struct PcgDev {
    double *rho, *pq, *alpha, *beta, *rn2, *bn2, *tol2;
    int *done, *brk, *iters;
    double *hist;   // rn2 per iteration, [hist_len][R], or null
    int hist_len;
    double *rzo;    // flexible beta: r'.z_old per column, or null (beta = rho'/rho)
};
void pcg_init_scalars(mm_ctx *ctx, int nrhs, PcgDev s, double tol);
void axpby_cols(mm_ctx *ctx, int64_t n, int nrhs, const double *b, const double *Ax, double *r);
// alpha from the p.q partials, then x += alpha p, r -= alpha q with the
// ||r||^2 partials (into a buffer other than pq_part)
void pcg_update_xr(mm_ctx *ctx, int64_t n, int nrhs, PcgDev s, const double *pq_part,
                   const double *p, const double *q, double *x, double *r, double *partial,
                   int n_part);
// breakdown flag, iteration count and convergence from ||r||^2, then rho', beta
void pcg_after_rnrz(mm_ctx *ctx, int nrhs, PcgDev s, const double *part_rn,
                    const double *part_rz, int n_part);
void pcg_after_rn(mm_ctx *ctx, int nrhs, PcgDev s, const double *partial, int n_part,
                  int count_iter);
void pcg_after_rz(mm_ctx *ctx, int nrhs, PcgDev s, const double *partial, int n_part, int init);
// s.rzo[r] = sum of the column's partial dot products (flexible beta)
void pcg_store_rzo(mm_ctx *ctx, int nrhs, PcgDev s, const double *partial, int n_part);
void pcg_update_p(mm_ctx *ctx, int64_t n, int nrhs, PcgDev s, const double *z, double *p);
void dot_partial_cols(mm_ctx *ctx, int64_t n, int nrhs, const double *a, const double *b,
                      double *partial, int n_part);
void col_set(mm_ctx *ctx, int64_t n, int R, int slot, const double *src, double *dst);
void gemm_rows_small(mm_ctx *ctx, int64_t n, int R, const double *In, const double *S,
                     double alpha, double beta, double *Out);
void chol_inv_drop(mm_ctx *ctx, int R, const double *G, double tau, double *U, int *rank);
void col_get(mm_ctx *ctx, int64_t n, int R, int slot, const double *src, double *dst);
// dst (k columns over the n_dst_obs pixels obs_dst) = src's rows of the same
// global pixels (k columns over obs_src), 0 where obs_src lacks the pixel
void transfer_rows(mm_ctx *ctx, int32_t n_dst_obs, const int32_t *obs_dst, int32_t n_src_obs,
                   const int32_t *obs_src, int nc, int k, const double *src, double *dst);
void slot_ctl(mm_ctx *ctx, PcgDev s, int slot, int mode, double tol);
void copy_cols_masked(mm_ctx *ctx, int64_t n, int nrhs, const int *done, const double *src,
                      double *dst);

// host
void hessenberg_eig(int m, const double *H, double *wr, double *wi, double *vr, double *vi);
// Eigen-decomposition of a small symmetric matrix (cyclic Jacobi rotations):
// A (n x n, row-major) is destroyed; w = eigenvalues, U column j = vector j.
void sym_eig_jacobi(int n, std::vector<double> &A, std::vector<double> &w, std::vector<double> &U);

template <typename T> struct Vec2T;
template <> struct Vec2T<float> { using type = float2; };
template <> struct Vec2T<double> { using type = double2; };

void build_band_tiles(mm_ctx *ctx, mm_noise *nz);
void autotune(mm_ctx *ctx, mm_pointing *p, mm_noise *nz, int nrhs, int flags, double *report,
              int *n_report, int max_report);

inline int log2i(int r) { int l = 0; while ((1 << l) < r) ++l; return l; }
inline int pow2_ok(int r) { return r >= 1 && r <= 64 && (r & (r - 1)) == 0; }

}  // namespace mm

// Error handling at the C-ABI boundary: an mm::Error (or a host allocation
// failure) inside API_BEGIN(ctx) ... API_END becomes the call's status and the
// context's last-error message.
#define API_BEGIN(ctxp)                                   \
    mm_ctx *api_ctx_ = (ctxp);                            \
    try {                                                 \
        if (api_ctx_) {                                   \
            api_ctx_->last_error.clear();                 \
            MM_HIP(hipSetDevice(api_ctx_->device));       \
        }

#define API_END                                                            \
    }                                                                      \
    catch (const mm::Error &e) {                                           \
        if (api_ctx_) api_ctx_->last_error = e.what();                     \
        return e.code;                                                     \
    }                                                                      \
    catch (const std::bad_alloc &) {                                       \
        if (api_ctx_) api_ctx_->last_error = "host allocation failed";     \
        return MM_E_OOM;                                                   \
    }                                                                      \
    catch (const std::exception &e) {                                      \
        if (api_ctx_) api_ctx_->last_error = e.what();                     \
        return MM_E_DEVICE;                                                \
    }

namespace mm {
// Looks up, once per device and with that device current, the device address
// of the static scratch array of mm_apply_A_noalloc (called at context
// creation).
void noalloc_init(int device);
}  // namespace mm
