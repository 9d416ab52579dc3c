// C-ABI entry points: argument validation, handle ownership, and the host
// control loops (PCG, Arnoldi) that drive the device kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstring>
#include <functional>
#include <numeric>

#include "mm_internal.h"

namespace mm {

// ------------------------------------------------------------ profiler

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    MM_HIP(hipEventCreate(&e));
    return e;
}

void Profiler::flush() {
    for (auto &p : pending) {
        MM_HIP(hipEventSynchronize(p.b));
        float ms = 0;
        MM_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        auto &st = stages[p.name];
        st.ms += ms;
        st.calls += 1;
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}

Profiler::~Profiler() {
    for (auto &p : pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

Scope::Scope(Profiler &p, hipStream_t st, const char *n) : pr(&p), s(st), name(n) {
    if (!pr->on) return;
    a = pr->get();
    b = pr->get();
    (void)hipEventRecord(a, s);
}

Scope::~Scope() {
    if (!pr->on) return;
    (void)hipEventRecord(b, s);
    pr->pending.push_back({name, a, b});
    if (pr->pending.size() > 4096) {
        try { pr->flush(); } catch (...) {}
    }
}


}  // namespace mm

using namespace mm;

namespace {

size_t tod_elem(mm_precision p) { return p == MM_F32 ? sizeof(float) : sizeof(double); }

void check_nrhs(int nrhs) {
    MM_CHECK(pow2_ok(nrhs), MM_E_INVALID, "nrhs must be 1, 2, 4, 8, 16, 32 or 64");
}

void check_pair(const mm_pointing *p, const mm_noise *nz) {
    MM_CHECK(p && nz, MM_E_INVALID, "null pointing or noise handle");
    MM_CHECK(p->n_samp == nz->n_samp, MM_E_INVALID,
             "pointing and noise cover different numbers of samples");
    MM_CHECK(p->prec == nz->prec, MM_E_INVALID, "pointing and noise precisions differ");
}

void ensure_tod(mm_ctx *ctx, const mm_pointing *p, int nrhs) {
    const size_t b = tod_elem(p->prec) * (size_t)p->n_samp * nrhs;
    ws_alloc(ctx, ctx->tod_a, b);
    ws_alloc(ctx, ctx->tod_b, b);
}

void apply_A_impl(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, int nrhs,
                  const double *x, double *y) {
    ensure_tod(ctx, p, nrhs);
    apply_P_dev(ctx, p, nrhs, x, ctx->tod_a.ptr);
    noise_apply_dev(ctx, nz, nrhs, ctx->tod_a.ptr, ctx->tod_b.ptr);
    apply_PT_dev(ctx, p, nrhs, ctx->tod_b.ptr, y);
}

double *pinned(mm_ctx *ctx, size_t bytes) {
    if (ctx->pinned_bytes < bytes) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        void *p = nullptr;
        MM_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
        ctx->pinned = static_cast<double *>(p);
        ctx->pinned_bytes = bytes;
    }
    return ctx->pinned;
}

void precond_apply_impl(mm_ctx *ctx, const mm_precond *M, int nrhs, const double *v, double *out,
                        double *partial, int n_part) {
    if (M->kind == 0)
        mbd_apply_dev(ctx, M->inv.as<double>(), M->n_obs, M->nc, nrhs, v, out, partial ? v : nullptr,
                      partial, n_part);
    else
        m2l_apply_dev(ctx, M, nrhs, v, out, partial, n_part);
}

// ||M r|| / ||M b|| per column (the residual of Eq. residuals read
// literally), into host out[R]; with M NULL, ||r|| / ||b||.  tmp: n R doubles.
void precond_rel_res(mm_ctx *ctx, const mm_precond *M, int64_t n, int R, const double *r,
                     const double *b, double *tmp, std::vector<double> &out) {
    DBuf d;
    d.alloc(sizeof(double) * 2 * R);
    const double *vr = r, *vb = b;
    if (M) {
        precond_apply_impl(ctx, M, R, r, tmp, nullptr, 0);
        vr = tmp;
    }
    dot_cols(ctx, n, R, vr, vr, d.as<double>());
    if (M) {
        precond_apply_impl(ctx, M, R, b, tmp, nullptr, 0);
        vb = tmp;
    }
    dot_cols(ctx, n, R, vb, vb, d.as<double>() + R);
    std::vector<double> h(2 * R);
    MM_HIP(hipMemcpyAsync(h.data(), d.ptr, sizeof(double) * 2 * R, hipMemcpyDeviceToHost,
                          ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
    out.resize(R);
    for (int c = 0; c < R; ++c)
        out[c] = h[R + c] > 0 ? std::sqrt(std::max(h[c], 0.0) / h[R + c]) : 0.0;
}

// The coarse part of M_2l once Z and AZ are on the device (column-major
// n x k): E = Z^T AZ, its Cholesky factor and from it E^-1.
static void finish_coarse(mm_ctx *ctx, int64_t n, mm_precond *M) {
    const int k = M->k;
    M->E.alloc(sizeof(double) * k * k);
    M->Einv.alloc(sizeof(double) * k * k);
    gram_mfma(ctx, n, k, k, M->Z.as<double>(), 1, n, M->AZ.as<double>(), 1, n, M->E.as<double>());
    DBuf flag, Lc;
    flag.alloc(sizeof(int));
    Lc.alloc(sizeof(double) * k * k);
    chol_small_dev(ctx, k, M->E.as<double>(), Lc.as<double>(), flag.as<int>());
    // formed before the pivot check (one wait for both); not used if it fails
    coarse_inverse_dev(ctx, k, Lc.as<double>(), M->Einv.as<double>());
    int hf = 0;
    MM_HIP(hipMemcpyAsync(&hf, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
    MM_CHECK(!hf, MM_E_COARSE_NOT_SPD, "coarse matrix E = Z^T A Z is not positive definite");
}

// M_2l from Z (device, column-major n x k): AZ by k applies of A, then the
// coarse part.
void finish_m2l(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, mm_precond *M) {
    const int64_t n = p->n();
    const int k = M->k;
    M->AZ.alloc(sizeof(double) * n * k);
    for (int c = 0; c < k; ++c)
        apply_A_impl(ctx, p, nz, 1, M->Z.as<double>() + (int64_t)c * n,
                     M->AZ.as<double>() + (int64_t)c * n);
    finish_coarse(ctx, n, M);
}

// Device vectors and scalars of a column-batched PCG (Eq. pcg).
struct PcgWork {
    int R = 1;
    int64_t n = 0;
    int n_part = 1;
    DBuf r, z, pv, q, part, part2, sc;  // part2: the ||r||^2 partials of an iteration
    PcgDev sd{};
    bool flexible = false;  // Polak-Ribiere beta (sd.rzo holds r'.z_old)
    void alloc(int64_t n_, int R_) {
        n = n_;
        R = R_;
        n_part = reduction_parts(n, R_);
        const size_t vb = sizeof(double) * n * R;
        r.alloc(vb);
        z.alloc(vb);
        pv.alloc(vb);
        q.alloc(vb);
        part.alloc(sizeof(double) * n_part * R);
        part2.alloc(sizeof(double) * n_part * R);
        sc.alloc(sizeof(double) * 8 * 64 + sizeof(int) * 3 * 64);
        double *sb = sc.as<double>();
        sd.rho = sb; sd.pq = sb + 64; sd.alpha = sb + 128; sd.beta = sb + 192;
        sd.rn2 = sb + 256; sd.bn2 = sb + 320; sd.tol2 = sb + 384;
        sd.rzo = flexible ? sb + 448 : nullptr;
        int *ib = reinterpret_cast<int *>(sb + 512);
        sd.done = ib; sd.brk = ib + 64; sd.iters = ib + 128;
        sd.hist = nullptr;
        sd.hist_len = 0;
    }
};

// A captured chunk of PCG iterations, replayed with one hipGraphLaunch.  The
// kernels of an iteration take only device-resident scalars, so the chunk is
// the same graph every time; finished columns turn every kernel into a no-op.
struct PcgGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    int chunk = 0;
    uint64_t gen = 0;  // context workspace generation the graph was captured with
    void reset() {
        if (ex) (void)hipGraphExecDestroy(ex);
        if (g) (void)hipGraphDestroy(g);
        ex = nullptr;
        g = nullptr;
    }
    // A graph whose workspaces have since been reallocated must be captured again.
    void drop_if_stale(const mm_ctx *ctx) {
        if (ex && gen != ctx->ws_gen) reset();
    }
    ~PcgGraph() { reset(); }
};

// z = M r on all columns with the fused partial sums of r.z.
void pcg_apply_M(mm_ctx *ctx, const mm_precond *M, PcgWork &w, const double *in, double *out) {
    if (M) {
        precond_apply_impl(ctx, M, w.R, in, out, w.part.as<double>(), w.n_part);
    } else {
        MM_HIP(hipMemcpyAsync(out, in, sizeof(double) * w.n * w.R, hipMemcpyDeviceToDevice,
                              ctx->stream));
        dot_partial_cols(ctx, w.n, w.R, in, out, w.part.as<double>(), w.n_part);
    }
}

// One lockstep iteration over the live columns:
//   q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q; ||r||^2;
//   z = M r; rho' = r.z; beta = rho'/rho; p = z + beta p.
// alpha is taken inside the x, r update, and the ||r||^2 test together with
// rho' and beta in one small launch after z = M r (its partials kept apart).
void pcg_iteration(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, const mm_precond *M,
                   PcgWork &w, double *x) {
    const int R = w.R;
    apply_A_impl(ctx, p, nz, R, w.pv.as<double>(), w.q.as<double>());
    dot_partial_cols(ctx, w.n, R, w.pv.as<double>(), w.q.as<double>(), w.part.as<double>(),
                     w.n_part);
    pcg_update_xr(ctx, w.n, R, w.sd, w.part.as<double>(), w.pv.as<double>(), w.q.as<double>(), x,
                  w.r.as<double>(), w.part2.as<double>(), w.n_part);
    if (w.flexible) {  // r'.z_old before z is overwritten
        dot_partial_cols(ctx, w.n, R, w.r.as<double>(), w.z.as<double>(), w.part.as<double>(),
                         w.n_part);
        pcg_store_rzo(ctx, R, w.sd, w.part.as<double>(), w.n_part);
    }
    pcg_apply_M(ctx, M, w, w.r.as<double>(), w.z.as<double>());
    pcg_after_rnrz(ctx, R, w.sd, w.part2.as<double>(), w.part.as<double>(), w.n_part);
    pcg_update_p(ctx, w.n, R, w.sd, w.z.as<double>(), w.pv.as<double>());
}

void capture_chunk(mm_ctx *ctx, PcgGraph &G, int chunk, const std::function<void()> &body) {
    if (!ctx->cap) MM_HIP(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    hipStream_t keep = ctx->stream;
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    ctx->stream = ctx->cap;
    hipError_t e = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        try {
            for (int i = 0; i < chunk; ++i) body();
        } catch (...) {
            hipGraph_t junk;
            (void)hipStreamEndCapture(ctx->cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            ctx->stream = keep;
            ctx->prof.on = prof;
            throw;
        }
        e = hipStreamEndCapture(ctx->cap, &G.g);
    }
    ctx->stream = keep;
    ctx->prof.on = prof;
    MM_HIP(e);
    MM_HIP(hipGraphInstantiate(&G.ex, G.g, nullptr, nullptr, 0));
    G.chunk = chunk;
    G.gen = ctx->ws_gen;
}


}  // namespace

// ================================================================ context

extern "C" const char *mm_version(void) { return "mapmaker-mi355x 0.1"; }

extern "C" mm_status mm_ctx_create(int device, void *hip_stream, mm_ctx **out) {
    if (!out) return MM_E_INVALID;
    *out = nullptr;
    mm_ctx *ctx = nullptr;
    try {
        int ndev = 0;
        MM_HIP(hipGetDeviceCount(&ndev));
        MM_CHECK(device >= 0 && device < ndev, MM_E_INVALID, "no such device");
        MM_HIP(hipSetDevice(device));
        ctx = new mm_ctx();
        ctx->device = device;
        if (hip_stream) {
            ctx->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            MM_HIP(hipStreamCreate(&ctx->stream));
            ctx->own_stream = true;
        }
        hipDeviceProp_t prop;
        MM_HIP(hipGetDeviceProperties(&prop, device));
        ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        noalloc_init(device);
        *out = ctx;
        return MM_OK;
    } catch (const mm::Error &e) {
        delete ctx;
        return e.code;
    } catch (...) {
        delete ctx;
        return MM_E_DEVICE;
    }
}

extern "C" void mm_ctx_destroy(mm_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
}

extern "C" const char *mm_last_error(const mm_ctx *ctx) {
    return ctx ? ctx->last_error.c_str() : "null context";
}

// =============================================================== pointing

extern "C" mm_status mm_pointing_build_stokes(mm_ctx *ctx, int64_t n_samp, int32_t n_pix_total,
                                              const int32_t *pix, const double *psi,
                                              int32_t min_hits, mm_precision prec,
                                              mm_stokes stokes, mm_pointing **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    MM_CHECK(n_samp > 0 && n_samp < ((int64_t)1 << 31), MM_E_INVALID,
             "n_samp must be in (0, 2^31)");
    MM_CHECK(n_pix_total > 0, MM_E_INVALID, "n_pix_total must be positive");
    MM_CHECK(stokes == MM_STOKES_IQU || stokes == MM_STOKES_I || stokes == MM_STOKES_QU,
             MM_E_INVALID, "stokes must be IQU, I or QU");
    MM_CHECK(pix && (psi || stokes == MM_STOKES_I), MM_E_INVALID, "null pix/psi");
    MM_CHECK(min_hits >= 1, MM_E_INVALID, "min_hits must be >= 1");
    MM_CHECK(prec == MM_F64 || prec == MM_F32, MM_E_INVALID, "bad precision");
    auto *p = new mm_pointing();
    p->n_samp = n_samp;
    p->n_pix_total = n_pix_total;
    p->prec = prec;
    p->stokes = stokes;
    p->nc = stokes == MM_STOKES_IQU ? 3 : stokes == MM_STOKES_QU ? 2 : 1;
    try {
        pointing_build_device(ctx, p, pix, stokes == MM_STOKES_I ? nullptr : psi, min_hits);
    } catch (...) {
        delete p;
        throw;
    }
    *out = p;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pointing_build(mm_ctx *ctx, int64_t n_samp, int32_t n_pix_total,
                                       const int32_t *pix, const double *psi, int32_t min_hits,
                                       mm_precision prec, mm_pointing **out) {
    return mm_pointing_build_stokes(ctx, n_samp, n_pix_total, pix, psi, min_hits, prec,
                                    MM_STOKES_IQU, out);
}

extern "C" mm_status mm_pointing_stokes(const mm_pointing *p, mm_stokes *stokes, int32_t *nc) {
    if (!p) return MM_E_INVALID;
    if (stokes) *stokes = p->stokes;
    if (nc) *nc = p->nc;
    return MM_OK;
}

extern "C" mm_status mm_pair_sum_diff(mm_ctx *ctx, int64_t n, mm_precision prec, const void *a,
                                      const void *b, void *plus, void *minus) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(n >= 0, MM_E_INVALID, "pair_sum_diff: negative length");
    MM_CHECK(prec == MM_F64 || prec == MM_F32, MM_E_INVALID, "bad precision");
    MM_CHECK(n == 0 || (a && b), MM_E_INVALID, "pair_sum_diff: null input");
    if (n > 0 && (plus || minus)) pair_sum_diff_dev(ctx, n, prec, a, b, plus, minus);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pointing_set_grid(mm_ctx *ctx, mm_pointing *p, int32_t width) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(p, MM_E_INVALID, "set_grid: null pointing");
    MM_CHECK(width >= 0, MM_E_INVALID, "set_grid: negative width");
    if (width == 0) {
        p->seg_order.release();
        p->grid_width = 0;
    } else {
        pointing_set_grid_device(ctx, p, width, 32);
        p->grid_width = width;
    }
    // P's map copies first: the sliced P^T is cut by the same scan directions
    pointing_p_slots_device(ctx, p, width);
    pointing_slices_device(ctx, p, width);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pointing_p_layout(const mm_pointing *p, int32_t *copies) {
    if (!p || !copies) return MM_E_INVALID;
    *copies = p->p_j.ptr ? p->p_copies : 0;
    return MM_OK;
}

extern "C" mm_status mm_pointing_pt_layout(const mm_pointing *p, int32_t *slices,
                                           int32_t *segments) {
    if (!p || !slices || !segments) return MM_E_INVALID;
    *slices = p->sl_G;
    *segments = p->sl_S;
    return MM_OK;
}

extern "C" mm_status mm_pointing_counts(const mm_pointing *p, int32_t *n_obs, int64_t *n_valid) {
    if (!p) return MM_E_INVALID;
    if (n_obs) *n_obs = p->n_obs;
    if (n_valid) *n_valid = p->n_valid;
    return MM_OK;
}

extern "C" mm_status mm_pointing_hits(mm_ctx *ctx, const mm_pointing *p, int32_t *hits,
                                      int32_t *obs_pix) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(p, MM_E_INVALID, "null pointing");
    if (hits)
        MM_HIP(hipMemcpyAsync(hits, p->hits.ptr, sizeof(int32_t) * p->n_pix_total,
                              hipMemcpyDeviceToDevice, ctx->stream));
    if (obs_pix && p->n_obs)
        MM_HIP(hipMemcpyAsync(obs_pix, p->obs_pix.ptr, sizeof(int32_t) * p->n_obs,
                              hipMemcpyDeviceToDevice, ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pointing_export(mm_ctx *ctx, const mm_pointing *p, int32_t *j,
                                        int32_t *perm, int32_t *off) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(p, MM_E_INVALID, "null pointing");
    if (j)
        MM_HIP(hipMemcpyAsync(j, p->j.ptr, sizeof(int32_t) * p->n_samp, hipMemcpyDeviceToDevice,
                              ctx->stream));
    if (perm && p->n_valid)
        MM_HIP(hipMemcpyAsync(perm, p->perm.ptr, sizeof(int32_t) * p->n_valid,
                              hipMemcpyDeviceToDevice, ctx->stream));
    if (off)
        MM_HIP(hipMemcpyAsync(off, p->off.ptr, sizeof(int32_t) * (p->n_obs + 1),
                              hipMemcpyDeviceToDevice, ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
    API_END
    return MM_OK;
}

extern "C" void mm_pointing_destroy(mm_pointing *p) { delete p; }

// ================================================================== noise

extern "C" mm_status mm_noise_build(mm_ctx *ctx, int32_t n_intervals,
                                    const int64_t *interval_start, const int32_t *filter_id,
                                    int32_t n_filters, int32_t half_bw, const double *band,
                                    mm_noise_method method, mm_precision prec, mm_noise **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    MM_CHECK(n_intervals > 0 && interval_start && filter_id && band, MM_E_INVALID,
             "noise: empty or null arguments");
    MM_CHECK(n_filters > 0 && half_bw >= 0, MM_E_INVALID, "noise: bad filter count or bandwidth");
    MM_CHECK(prec == MM_F64 || prec == MM_F32, MM_E_INVALID, "bad precision");
    MM_CHECK(interval_start[0] == 0, MM_E_INVALID, "intervals must start at sample 0");
    int64_t min_len = INT64_MAX;
    for (int i = 0; i < n_intervals; ++i) {
        const int64_t L = interval_start[i + 1] - interval_start[i];
        MM_CHECK(L > 0, MM_E_INVALID, "intervals must be strictly increasing");
        min_len = std::min(min_len, L);
        MM_CHECK(filter_id[i] >= 0 && filter_id[i] < n_filters, MM_E_INVALID,
                 "filter id out of range");
    }
    MM_CHECK(2 * (int64_t)half_bw < min_len, MM_E_INVALID,
             "half bandwidth must be below half the shortest interval");
    MM_CHECK(interval_start[n_intervals] < ((int64_t)1 << 31), MM_E_INVALID, "too many samples");
    const size_t nb = (size_t)n_filters * (half_bw + 1);
    for (size_t i = 0; i < nb; ++i)
        MM_CHECK(std::isfinite(band[i]), MM_E_NONFINITE, "non-finite band coefficient");
    MM_CHECK(method == MM_NOISE_AUTO || method == MM_NOISE_DIRECT || method == MM_NOISE_FFT,
             MM_E_INVALID, "bad noise method");

    auto *nz = new mm_noise();
    try {
        nz->n_samp = interval_start[n_intervals];
        nz->n_int = n_intervals;
        nz->n_filters = n_filters;
        nz->half_bw = half_bw;
        nz->prec = prec;
        nz->h_istart.assign(interval_start, interval_start + n_intervals + 1);
        nz->h_fid.assign(filter_id, filter_id + n_intervals);
        nz->h_band.assign(band, band + nb);
        const bool fft_ok = noise_fft_supported(half_bw, min_len);
        if (method == MM_NOISE_FFT) {
            MM_CHECK(fft_ok, MM_E_INVALID, "FFT noise method unsupported for this bandwidth");
            nz->method = MM_NOISE_FFT;
        } else if (method == MM_NOISE_AUTO) {
            // measured crossover (direct band vs overlap-save FFT, FP64,
            // 2^20..2^27 samples in 2^16-sample intervals): on streams of 2^22
            // samples and more the FFT wins from lambda = 32 on (its time
            // hardly depends on lambda, the band's grows with it); on shorter
            // ones from 128.  FP32 keeps the earlier crossover at 64.
            const bool long_stream = nz->n_samp >= ((int64_t)1 << 22);
            const int cross = long_stream ? (prec == MM_F64 ? 32 : 64) : 128;
            nz->method = (fft_ok && half_bw >= cross) ? MM_NOISE_FFT : MM_NOISE_DIRECT;
        } else {
            nz->method = MM_NOISE_DIRECT;
        }
        hipStream_t s = ctx->stream;
        nz->istart.alloc(sizeof(int64_t) * (n_intervals + 1));
        nz->fid.alloc(sizeof(int32_t) * n_intervals);
        nz->band64.alloc(sizeof(double) * nb);
        MM_HIP(hipMemcpyAsync(nz->istart.ptr, interval_start, sizeof(int64_t) * (n_intervals + 1),
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipMemcpyAsync(nz->fid.ptr, filter_id, sizeof(int32_t) * n_intervals,
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipMemcpyAsync(nz->band64.ptr, band, sizeof(double) * nb, hipMemcpyHostToDevice, s));
        if (prec == MM_F32) {
            std::vector<float> bf(band, band + nb);
            nz->band.alloc(sizeof(float) * nb);
            MM_HIP(hipMemcpyAsync(nz->band.ptr, bf.data(), sizeof(float) * nb,
                                  hipMemcpyHostToDevice, s));
            MM_HIP(hipStreamSynchronize(s));
        } else {
            nz->band.alloc(sizeof(double) * nb);
            MM_HIP(hipMemcpyAsync(nz->band.ptr, band, sizeof(double) * nb,
                                  hipMemcpyHostToDevice, s));
        }
        // direct-band tile counts for every column count, built here so that
        // applies never modify the handle; one column on a short stream is
        // cut into small tiles so that it still fills the CUs
        nz->band_small = nz->n_samp <= (int64_t(1) << 20);
        build_band_tiles(ctx, nz);
        if (nz->method == MM_NOISE_FFT) noise_fft_prepare(ctx, nz, 0);
    } catch (...) {
        delete nz;
        throw;
    }
    *out = nz;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_polyfilter_build(mm_ctx *ctx, const mm_pointing *p, int32_t n_intervals,
                                         const int64_t *interval_start, const double *weight,
                                         int64_t n_subscans, const int64_t *subscan_start,
                                         int32_t order, const int32_t *ground_bin,
                                         int32_t n_ground_bins, mm_noise **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    MM_CHECK(p, MM_E_INVALID, "polyfilter: null pointing");
    MM_CHECK(n_intervals > 0 && interval_start && weight && n_subscans > 0 && subscan_start,
             MM_E_INVALID, "polyfilter: empty or null arguments");
    MM_CHECK(order >= 0 && order <= polyfilter_max_order(), MM_E_INVALID,
             "polyfilter: order must be in [0, 7]");
    MM_CHECK(ground_bin ? n_ground_bins >= 1 : n_ground_bins == 0, MM_E_INVALID,
             "polyfilter: ground bins need n_ground_bins >= 1 (0 without them)");
    const int64_t n = p->n_samp;
    MM_CHECK(interval_start[0] == 0 && interval_start[n_intervals] == n, MM_E_INVALID,
             "polyfilter: intervals must tile [0, n_samp)");
    for (int i = 0; i < n_intervals; ++i) {
        MM_CHECK(interval_start[i + 1] > interval_start[i], MM_E_INVALID,
                 "polyfilter: intervals must be strictly increasing");
        MM_CHECK(std::isfinite(weight[i]), MM_E_NONFINITE, "polyfilter: non-finite weight");
        MM_CHECK(weight[i] >= 0, MM_E_INVALID, "polyfilter: negative weight");
    }
    MM_CHECK(subscan_start[0] == 0 && subscan_start[n_subscans] == n, MM_E_INVALID,
             "polyfilter: subscans must tile [0, n_samp)");
    std::vector<double> om((size_t)n_subscans);
    int iv = 0;
    int64_t max_len = 0;
    for (int64_t s2 = 0; s2 < n_subscans; ++s2) {
        const int64_t a = subscan_start[s2], b = subscan_start[s2 + 1];
        MM_CHECK(b > a, MM_E_INVALID, "polyfilter: subscans must be strictly increasing");
        max_len = std::max(max_len, b - a);
        while (interval_start[iv + 1] <= a) ++iv;
        MM_CHECK(b <= interval_start[iv + 1], MM_E_INVALID,
                 "polyfilter: a subscan crosses an interval boundary");
        om[(size_t)s2] = weight[iv];
    }
    auto *nz = new mm_noise();
    try {
        nz->n_samp = n;
        nz->n_int = n_intervals;
        nz->n_filters = n_intervals;
        nz->half_bw = 0;
        nz->prec = p->prec;
        nz->method = MM_NOISE_POLY;
        nz->pf_max_len = max_len;
        nz->h_istart.assign(interval_start, interval_start + n_intervals + 1);
        nz->h_fid.resize(n_intervals);
        std::iota(nz->h_fid.begin(), nz->h_fid.end(), 0);
        nz->h_band.assign(weight, weight + n_intervals);
        hipStream_t s = ctx->stream;
        nz->istart.alloc(sizeof(int64_t) * (n_intervals + 1));
        nz->fid.alloc(sizeof(int32_t) * n_intervals);
        nz->band64.alloc(sizeof(double) * n_intervals);
        MM_HIP(hipMemcpyAsync(nz->istart.ptr, interval_start, sizeof(int64_t) * (n_intervals + 1),
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipMemcpyAsync(nz->fid.ptr, nz->h_fid.data(), sizeof(int32_t) * n_intervals,
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipMemcpyAsync(nz->band64.ptr, weight, sizeof(double) * n_intervals,
                              hipMemcpyHostToDevice, s));
        nz->pf_order = order;
        nz->pf_n_sub = n_subscans;
        nz->pf_sub.alloc(sizeof(int64_t) * (n_subscans + 1));
        nz->pf_omega.alloc(sizeof(double) * n_subscans);
        MM_HIP(hipMemcpyAsync(nz->pf_sub.ptr, subscan_start, sizeof(int64_t) * (n_subscans + 1),
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipMemcpyAsync(nz->pf_omega.ptr, om.data(), sizeof(double) * n_subscans,
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipStreamSynchronize(s));
        polyfilter_prepare(ctx, p, nz, ground_bin, n_ground_bins);
    } catch (...) {
        delete nz;
        throw;
    }
    *out = nz;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_noise_method_used(const mm_noise *nz, mm_noise_method *method) {
    if (!nz || !method) return MM_E_INVALID;
    *method = nz->method;
    return MM_OK;
}

extern "C" mm_status mm_noise_fft_block(const mm_noise *nz, int32_t *n_fft, int32_t *n_valid) {
    if (!nz || !n_fft || !n_valid) return MM_E_INVALID;
    const bool fft = nz->method == MM_NOISE_FFT;
    *n_fft = fft ? (int32_t)nz->fft_n : 0;
    *n_valid = fft ? (int32_t)nz->fft_valid : 0;
    return MM_OK;
}

extern "C" mm_status mm_noise_set_fft_block(mm_ctx *ctx, mm_noise *nz, int32_t n_fft) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(nz && nz->method == MM_NOISE_FFT, MM_E_INVALID,
             "noise_set_fft_block: needs a noise handle applied by FFT");
    MM_CHECK(n_fft >= 0, MM_E_INVALID, "noise_set_fft_block: negative block length");
    MM_HIP(hipStreamSynchronize(ctx->stream));
    noise_fft_prepare(ctx, nz, n_fft);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_noise_apply(mm_ctx *ctx, const mm_noise *nz, int32_t nrhs, const void *y,
                                    void *z) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(nz && y && z && y != z, MM_E_INVALID, "noise apply: bad arguments");
    check_nrhs(nrhs);
    noise_apply_dev(ctx, nz, nrhs, y, z);
    API_END
    return MM_OK;
}

extern "C" void mm_noise_destroy(mm_noise *nz) { delete nz; }

// ============================================================== operators

extern "C" mm_status mm_apply_P(mm_ctx *ctx, const mm_pointing *p, int32_t nrhs, const double *x,
                                void *y) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(p && x && y, MM_E_INVALID, "apply_P: null argument");
    check_nrhs(nrhs);
    apply_P_dev(ctx, p, nrhs, x, y);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_apply_PT(mm_ctx *ctx, const mm_pointing *p, int32_t nrhs, const void *z,
                                 double *x) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(p && x && z, MM_E_INVALID, "apply_PT: null argument");
    check_nrhs(nrhs);
    apply_PT_dev(ctx, p, nrhs, z, x);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_apply_A(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                int32_t nrhs, const double *x, double *y) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    check_pair(p, nz);
    MM_CHECK(x && y && x != y, MM_E_INVALID, "apply_A: x and y must be distinct and non-null");
    check_nrhs(nrhs);
    apply_A_impl(ctx, p, nz, nrhs, x, y);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_rhs(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, int32_t nrhs,
                            const void *tod, double *b) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    check_pair(p, nz);
    MM_CHECK(tod && b, MM_E_INVALID, "rhs: null argument");
    check_nrhs(nrhs);
    ensure_tod(ctx, p, nrhs);
    DBuf flag;
    flag.alloc(sizeof(int));
    MM_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), ctx->stream));
    mask_tod_dev(ctx, p, nrhs, tod, ctx->tod_a.ptr, flag.as<int>());
    int hf = 0;
    MM_HIP(hipMemcpyAsync(&hf, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
    MM_CHECK(!hf, MM_E_NONFINITE, "rhs: non-finite TOD sample on an observed pixel");
    noise_apply_dev(ctx, nz, nrhs, ctx->tod_a.ptr, ctx->tod_b.ptr);
    apply_PT_dev(ctx, p, nrhs, ctx->tod_b.ptr, b);
    API_END
    return MM_OK;
}

// ======================================================== preconditioners

extern "C" mm_status mm_mbd_build(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                  mm_precond **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    check_pair(p, nz);
    auto *M = new mm_precond();
    M->kind = 0;
    M->n_obs = p->n_obs;
    M->nc = p->nc;
    int bad = 0;
    try {
        mbd_build_dev(ctx, p, nz, M, &bad);
    } catch (...) {
        delete M;
        throw;
    }
    if (bad) {
        delete M;
        throw Error(MM_E_SINGULAR_BLOCK,
                    std::to_string(bad) + " pixel block(s) singular or with rcond < 1e-12");
    }
    *out = M;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_mbd_rcond(const mm_precond *M, double *rcond_min) {
    if (!M || !rcond_min) return MM_E_INVALID;
    *rcond_min = M->rcond_min;
    return MM_OK;
}

extern "C" mm_status mm_defl_from_Z(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                    const mm_precond *mbd, int32_t k, const double *Z,
                                    mm_precond **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    check_pair(p, nz);
    MM_CHECK(mbd && mbd->kind == 0 && mbd->n_obs == p->n_obs && mbd->nc == p->nc, MM_E_INVALID,
             "defl: needs an M_BD handle of the same pointing");
    MM_CHECK(k >= 1 && k <= 64 && k <= p->n(), MM_E_INVALID, "defl: k must be in [1, 64]");
    MM_CHECK(Z, MM_E_INVALID, "defl: null Z");
    const int64_t n = p->n();
    auto *M = new mm_precond();
    try {
        M->kind = 1;
        M->n_obs = p->n_obs;
    M->nc = p->nc;
        M->k = k;
        M->rcond_min = mbd->rcond_min;
        M->inv.alloc(sizeof(double) * packed_sym(p->nc) * p->n_obs);
        MM_HIP(hipMemcpyAsync(M->inv.ptr, mbd->inv.ptr, sizeof(double) * packed_sym(p->nc) * p->n_obs,
                              hipMemcpyDeviceToDevice, ctx->stream));
        M->Z.alloc(sizeof(double) * n * k);
        MM_HIP(hipMemcpyAsync(M->Z.ptr, Z, sizeof(double) * n * k, hipMemcpyDeviceToDevice,
                              ctx->stream));
        finish_m2l(ctx, p, nz, M);
    } catch (...) {
        delete M;
        throw;
    }
    *out = M;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_defl_transfer(mm_ctx *ctx, const mm_pointing *p_src,
                                      const mm_precond *src, const mm_pointing *p,
                                      const mm_noise *nz, const mm_precond *mbd,
                                      mm_precond **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    check_pair(p, nz);
    MM_CHECK(p_src && src && src->kind == 1 && src->n_obs == p_src->n_obs && src->nc == p_src->nc,
             MM_E_INVALID, "defl_transfer: needs an M_2l handle of the source pointing");
    MM_CHECK(p_src->nc == p->nc, MM_E_INVALID, "defl_transfer: Stokes components differ");
    MM_CHECK(mbd && mbd->kind == 0 && mbd->n_obs == p->n_obs && mbd->nc == p->nc, MM_E_INVALID,
             "defl_transfer: needs an M_BD handle of the target pointing");
    const int k = src->k;
    const int64_t n = p->n();
    MM_CHECK(k >= 1 && k <= n, MM_E_INVALID, "defl_transfer: k exceeds the target's unknowns");
    auto *M = new mm_precond();
    try {
        M->kind = 1;
        M->n_obs = p->n_obs;
        M->nc = p->nc;
        M->k = k;
        M->rcond_min = mbd->rcond_min;
        M->inv.alloc(sizeof(double) * packed_sym(p->nc) * p->n_obs);
        MM_HIP(hipMemcpyAsync(M->inv.ptr, mbd->inv.ptr, sizeof(double) * packed_sym(p->nc) * p->n_obs,
                              hipMemcpyDeviceToDevice, ctx->stream));
        M->Z.alloc(sizeof(double) * n * k);
        transfer_rows(ctx, p->n_obs, p->obs_pix.as<int32_t>(), p_src->n_obs,
                      p_src->obs_pix.as<int32_t>(), p->nc, k, src->Z.as<double>(),
                      M->Z.as<double>());
        finish_m2l(ctx, p, nz, M);
    } catch (...) {
        delete M;
        throw;
    }
    *out = M;
    API_END
    return MM_OK;
}

// Ritz pairs of the m x m projected matrix Hm (column-major; Arnoldi's
// Hessenberg H_m or the Lanczos tridiagonal T_m), selection of the k smallest
// past the null directions (or all with Re theta < eps_lambda), V = W Y and
// Cholesky-QR twice: M->Z (n x kk, orthonormal) and M->k.  Then AZ, E.
// With drop_dependent, directions of V that are numerically dependent (an
// eigenvalue of V^T V below 1e-12 of the largest; finite-precision Lanczos
// repeats converged Ritz values) are left out before the Cholesky-QR, and kk
// shrinks accordingly; otherwise a dependent V is an error.
// AZ from the Arnoldi factorisation (App. A, Eq. factoriz) instead of k
// applies of A.  With B = M_BD A, B W_m = W_m H_m + r e_m^T, where r =
// h_{m+1,m} w_{m+1} is the last orthogonalised vector before normalisation,
// so A W_m = M_BD^-1 (W_m H_m + r e_m^T).  Z = W_m Y T (Y the selected Ritz
// vectors of H_m, T the orthonormalisation), hence
//   AZ = M_BD^-1 (W_m (H_m Y T) + r (e_m^T Y T)),
// one m x k product on the tall basis and, per column, M_BD^-1: the
// assembled 3 x 3 (or smaller) blocks blk.  Hbar is the (m+1) x m Hessenberg
// matrix (column-major), YT = Y T (m x k, column-major).
static void az_from_arnoldi(mm_ctx *ctx, mm_precond *M, const double *W, int m,
                            const std::vector<double> &Hbar, const std::vector<double> &YT,
                            int kk, const double *r, const double *blk) {
    hipStream_t s = ctx->stream;
    const int64_t n = M->n();
    std::vector<double> G((size_t)m * kk), g((size_t)kk);
    for (int c = 0; c < kk; ++c) {
        for (int i = 0; i < m; ++i) {
            double acc = 0;
            for (int j = 0; j < m; ++j) acc += Hbar[(size_t)j * (m + 1) + i] * YT[(size_t)c * m + j];
            G[(size_t)c * m + i] = acc;
        }
        g[(size_t)c] = YT[(size_t)c * m + (m - 1)];
    }
    DBuf Gd, gd, U;
    Gd.alloc(sizeof(double) * G.size());
    gd.alloc(sizeof(double) * g.size());
    MM_HIP(hipMemcpyAsync(Gd.ptr, G.data(), sizeof(double) * G.size(), hipMemcpyHostToDevice, s));
    MM_HIP(hipMemcpyAsync(gd.ptr, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, s));
    U.alloc(sizeof(double) * n * kk);
    matmul_small_right(ctx, n, m, kk, W, Gd.as<double>(), U.as<double>());
    rank1_add(ctx, n, kk, r, gd.as<double>(), U.as<double>());
    M->AZ.alloc(sizeof(double) * n * kk);
    for (int c = 0; c < kk; ++c)
        mbd_apply_dev(ctx, blk, M->n_obs, M->nc, 1, U.as<double>() + (int64_t)c * n,
                      M->AZ.as<double>() + (int64_t)c * n, nullptr, nullptr, 0);
    MM_HIP(hipStreamSynchronize(s));  // G and g are host vectors of this frame
}

// arn_res and blk given (an Arnoldi build): AZ from the factorisation
// (az_from_arnoldi); otherwise by applies of A.
static void z_from_ritz(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, mm_precond *M,
                        const double *W, int m, std::vector<double> &Hm, int k,
                        double eps_lambda, double *theta_out, bool drop_dependent = false,
                        const double *arn_res = nullptr, const double *blk = nullptr) {
    hipStream_t s = ctx->stream;
    const int64_t n = p->n();
    std::vector<double> wr(m), wi(m), vr((size_t)m * m), vi((size_t)m * m);
    hessenberg_eig(m, Hm.data(), wr.data(), wi.data(), vr.data(), vi.data());
    if (theta_out)
        for (int i = 0; i < m; ++i) theta_out[i] = wr[i];
    // Ritz values at the rounding level (|theta| <= 1e-10 max |theta|) are
    // exact null directions of M_BD A (sky modes a filter leaves
    // unconstrained): E could not be inverted with them, and a consistent
    // right-hand side has no component along them.  They stay out of Z.
    double tmax = 0;
    for (int i = 0; i < m; ++i) tmax = std::max(tmax, std::hypot(wr[i], wi[i]));
    int first = 0;
    while (first < m && std::hypot(wr[first], wi[first]) <= 1e-10 * tmax) ++first;
    int keep;
    if (eps_lambda > 0) {
        keep = 0;
        while (keep < m && wr[keep] < eps_lambda) ++keep;
    } else {
        keep = std::min(first + k, m);
    }
    auto pair_at = [&](int i) { return i + 1 < m && wi[i] != 0 && wi[i] == -wi[i + 1] && wr[i] == wr[i + 1]; };
    if (keep > 0 && keep < m && wi[keep - 1] != 0 && pair_at(keep - 1)) ++keep;
    std::vector<double> Y;
    int kk = 0;
    for (int i = first; i < keep && kk < 64;) {
        if (pair_at(i)) {
            if (kk + 2 > 64) break;
            Y.insert(Y.end(), vr.begin() + (size_t)i * m, vr.begin() + (size_t)(i + 1) * m);
            Y.insert(Y.end(), vi.begin() + (size_t)i * m, vi.begin() + (size_t)(i + 1) * m);
            kk += 2;
            i += 2;
        } else {
            Y.insert(Y.end(), vr.begin() + (size_t)i * m, vr.begin() + (size_t)(i + 1) * m);
            kk += 1;
            i += 1;
        }
    }
    MM_CHECK(kk >= 1, MM_E_INVALID, "defl: no Ritz vector selected");
    // T (column-major, kk0 x kk): Z = W_m Y T, accumulated over the steps below
    const int kk0 = kk;
    std::vector<double> T((size_t)kk0 * kk0, 0.0);
    for (int i = 0; i < kk0; ++i) T[(size_t)i * kk0 + i] = 1.0;
    auto t_times = [&](const std::vector<double> &Rm, int kin, int kout) {
        std::vector<double> nt((size_t)kk0 * kout, 0.0);
        for (int c = 0; c < kout; ++c)
            for (int q = 0; q < kin; ++q) {
                const double f = Rm[(size_t)c * kin + q];
                if (f == 0) continue;
                for (int r2 = 0; r2 < kk0; ++r2) nt[(size_t)c * kk0 + r2] += T[(size_t)q * kk0 + r2] * f;
            }
        T.swap(nt);
    };
    // V = W_m Y, then Cholesky-QR applied twice for an orthonormal Z
    DBuf Yd, V, G;
    Yd.alloc(sizeof(double) * Y.size());
    MM_HIP(hipMemcpyAsync(Yd.ptr, Y.data(), sizeof(double) * Y.size(), hipMemcpyHostToDevice, s));
    V.alloc(sizeof(double) * n * kk);
    M->Z.alloc(sizeof(double) * n * kk);
    matmul_small_right(ctx, n, m, kk, W, Yd.as<double>(), V.as<double>());
    G.alloc(sizeof(double) * kk * kk);
    if (drop_dependent) {
        // V <- V U_keep Lambda_keep^-1/2 (orthonormal up to rounding), into Z then back
        gram_mfma(ctx, n, kk, kk, V.as<double>(), 1, n, V.as<double>(), 1, n, G.as<double>());
        std::vector<double> g0((size_t)kk * kk), lam, U;
        MM_HIP(hipMemcpyAsync(g0.data(), G.ptr, sizeof(double) * kk * kk, hipMemcpyDeviceToHost, s));
        MM_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < kk; ++i)
            for (int j = 0; j < i; ++j)
                g0[(size_t)i * kk + j] = g0[(size_t)j * kk + i] =
                    0.5 * (g0[(size_t)i * kk + j] + g0[(size_t)j * kk + i]);
        sym_eig_jacobi(kk, g0, lam, U);
        double lmax = 0;
        for (double l : lam) lmax = std::max(lmax, l);
        std::vector<double> S;  // column-major kk x kk2
        int kk2 = 0;
        for (int j = 0; j < kk; ++j) {
            if (!(lam[j] > 1e-12 * lmax)) continue;
            const double sc = 1.0 / std::sqrt(lam[j]);
            for (int i = 0; i < kk; ++i) S.push_back(U[(size_t)i * kk + j] * sc);
            ++kk2;
        }
        MM_CHECK(kk2 >= 1, MM_E_COARSE_NOT_SPD, "defl: no independent Ritz vector");
        DBuf Sd;
        Sd.alloc(sizeof(double) * S.size());
        MM_HIP(hipMemcpyAsync(Sd.ptr, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice, s));
        matmul_small_right(ctx, n, kk, kk2, V.as<double>(), Sd.as<double>(), M->Z.as<double>());
        MM_HIP(hipMemcpyAsync(V.ptr, M->Z.ptr, sizeof(double) * n * kk2, hipMemcpyDeviceToDevice, s));
        MM_HIP(hipStreamSynchronize(s));
        t_times(S, kk, kk2);
        kk = kk2;
    }
    std::vector<double> g((size_t)kk * kk), rinv((size_t)kk * kk);
    for (int pass = 0; pass < 2; ++pass) {
        double *src = pass == 0 ? V.as<double>() : M->Z.as<double>();
        double *dst = pass == 0 ? M->Z.as<double>() : V.as<double>();
        gram_mfma(ctx, n, kk, kk, src, 1, n, src, 1, n, G.as<double>());
        MM_HIP(hipMemcpyAsync(g.data(), G.ptr, sizeof(double) * kk * kk, hipMemcpyDeviceToHost, s));
        MM_HIP(hipStreamSynchronize(s));
        // upper Cholesky factor R (G = R^T R), then R^-1 (column-major for the kernel)
        std::vector<double> R((size_t)kk * kk, 0.0);
        for (int c = 0; c < kk; ++c) {
            for (int r2 = 0; r2 <= c; ++r2) {
                double sum = 0.5 * (g[(size_t)r2 * kk + c] + g[(size_t)c * kk + r2]);
                for (int q = 0; q < r2; ++q) sum -= R[(size_t)q * kk + r2] * R[(size_t)q * kk + c];
                if (r2 == c) {
                    MM_CHECK(sum > 0, MM_E_COARSE_NOT_SPD, "defl: Ritz vectors linearly dependent");
                    R[(size_t)c * kk + c] = std::sqrt(sum);
                } else {
                    R[(size_t)r2 * kk + c] = sum / R[(size_t)r2 * kk + r2];
                }
            }
        }
        std::fill(rinv.begin(), rinv.end(), 0.0);
        for (int c = 0; c < kk; ++c) {  // solve R x = e_c
            std::vector<double> x(kk, 0.0);
            for (int r2 = c; r2 >= 0; --r2) {
                double sum = (r2 == c) ? 1.0 : 0.0;
                for (int q = r2 + 1; q <= c; ++q) sum -= R[(size_t)r2 * kk + q] * x[q];
                x[r2] = sum / R[(size_t)r2 * kk + r2];
            }
            for (int r2 = 0; r2 < kk; ++r2) rinv[(size_t)c * kk + r2] = x[r2];
        }
        MM_HIP(hipMemcpyAsync(G.ptr, rinv.data(), sizeof(double) * kk * kk, hipMemcpyHostToDevice, s));
        matmul_small_right(ctx, n, kk, kk, src, G.as<double>(), dst);
        MM_HIP(hipStreamSynchronize(s));
        t_times(rinv, kk, kk);
    }
    // after two passes the orthonormal basis is in V
    std::swap(M->Z, V);
    M->k = kk;
    if (arn_res && blk) {
        std::vector<double> YT((size_t)m * kk, 0.0);
        for (int c = 0; c < kk; ++c)
            for (int q = 0; q < kk0; ++q) {
                const double f = T[(size_t)c * kk0 + q];
                for (int r2 = 0; r2 < m; ++r2) YT[(size_t)c * m + r2] += Y[(size_t)q * m + r2] * f;
            }
        az_from_arnoldi(ctx, M, W, m, M->H, YT, kk, arn_res, blk);
        finish_coarse(ctx, n, M);
    } else {
        finish_m2l(ctx, p, nz, M);
    }
}

extern "C" mm_status mm_defl_build(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                   const mm_precond *mbd, const double *b_seed, int32_t k,
                                   double eps_lambda, double eps_arn, int32_t m_max,
                                   double *h_history, mm_arnoldi_info *info, mm_precond **out) {
    return mm_defl_build_stop(ctx, p, nz, mbd, b_seed, k, eps_lambda, eps_arn, MM_ARN_STOP_H,
                              m_max, h_history, nullptr, info, out);
}

extern "C" mm_status mm_defl_build_stop(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                        const mm_precond *mbd, const double *b_seed, int32_t k,
                                        double eps_lambda, double eps_arn, int32_t stop_rule,
                                        int32_t m_max, double *h_history, double *res_history,
                                        mm_arnoldi_info *info, mm_precond **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    auto t_start = std::chrono::steady_clock::now();
    check_pair(p, nz);
    MM_CHECK(stop_rule == MM_ARN_STOP_H || stop_rule == MM_ARN_STOP_RESIDUAL, MM_E_INVALID,
             "defl: unknown Arnoldi stop rule");
    MM_CHECK(mbd && mbd->kind == 0 && mbd->n_obs == p->n_obs && mbd->nc == p->nc, MM_E_INVALID,
             "defl: needs an M_BD handle of the same pointing");
    MM_CHECK(b_seed, MM_E_INVALID, "defl: null b_seed");
    const int64_t n = p->n();
    MM_CHECK(m_max >= 1 && m_max <= 500 && m_max <= n, MM_E_INVALID, "defl: m_max in [1, min(500, n)]");
    MM_CHECK(eps_lambda > 0 || (k >= 1 && k <= 63 && k <= m_max), MM_E_INVALID,
             "defl: k in [1, 63] and <= m_max");
    hipStream_t s = ctx->stream;
    auto *M = new mm_precond();
    try {
        M->kind = 1;
        M->n_obs = p->n_obs;
    M->nc = p->nc;
        M->rcond_min = mbd->rcond_min;
        M->inv.alloc(sizeof(double) * packed_sym(p->nc) * p->n_obs);
        MM_HIP(hipMemcpyAsync(M->inv.ptr, mbd->inv.ptr, sizeof(double) * packed_sym(p->nc) * p->n_obs,
                              hipMemcpyDeviceToDevice, s));
        M->W.alloc(sizeof(double) * n * (m_max + 1));
        double *W = M->W.as<double>();
        DBuf tmp, v, hd;
        tmp.alloc(sizeof(double) * n);
        v.alloc(sizeof(double) * n);
        hd.alloc(sizeof(double) * 1024);
        double *hp = pinned(ctx, sizeof(double) * 1024);
        // w_1 = r_0 / ||r_0||, r_0 = M_BD b
        mbd_apply_dev(ctx, M->inv.as<double>(), p->n_obs, p->nc, 1, b_seed, v.as<double>(), nullptr,
                      nullptr, 0);
        dot_cols(ctx, n, 1, v.as<double>(), v.as<double>(), hd.as<double>());
        MM_HIP(hipMemcpyAsync(hp, hd.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
        MM_HIP(hipStreamSynchronize(s));
        MM_CHECK(hp[0] > 0 && std::isfinite(hp[0]), MM_E_INVALID, "defl: zero start vector");
        const double nrm0 = std::sqrt(hp[0]);
        hp[1] = nrm0;
        MM_HIP(hipMemcpyAsync(hd.as<double>() + 1, hp + 1, sizeof(double), hipMemcpyHostToDevice, s));
        scale_copy(ctx, n, v.as<double>(), hd.as<double>() + 1, W, 1);
        std::vector<double> H((size_t)(m_max + 1) * m_max, 0.0);
        // Givens rotations reducing the (j+1) x j Hessenberg matrix to
        // triangular form: the least-squares residual after step j is
        // |gamma| = |s_1 ... s_j| (relative to ||r_0||) and the Arnoldi
        // (Galerkin) solution's residual h_{j+1,j} |(H_j^-1 e_1)_j| equals
        // |gamma| / |c_j| (Saad, Iterative Methods for Sparse Linear
        // Systems, 2nd ed., Sect. 6.5.7), so each step costs O(j)
        std::vector<double> gc(m_max), gs(m_max), col(m_max + 1);
        double gamma = 1.0;
        int m = 0;
        double h_last = 0;
        for (int j = 0; j < m_max; ++j) {
            const double *wj = W + (int64_t)j * n;
            apply_A_impl(ctx, p, nz, 1, wj, tmp.as<double>());
            mbd_apply_dev(ctx, M->inv.as<double>(), p->n_obs, p->nc, 1, tmp.as<double>(),
                          v.as<double>(), nullptr, nullptr, 0);
            // classical Gram-Schmidt, applied twice
            gemv_t(ctx, n, j + 1, W, v.as<double>(), hd.as<double>());
            gemv_n_sub(ctx, n, j + 1, W, hd.as<double>(), v.as<double>());
            gemv_t(ctx, n, j + 1, W, v.as<double>(), hd.as<double>() + 512);
            gemv_n_sub(ctx, n, j + 1, W, hd.as<double>() + 512, v.as<double>());
            dot_cols(ctx, n, 1, v.as<double>(), v.as<double>(), hd.as<double>() + 1023);
            MM_HIP(hipMemcpyAsync(hp, hd.ptr, sizeof(double) * 1024, hipMemcpyDeviceToHost, s));
            MM_HIP(hipStreamSynchronize(s));
            for (int i = 0; i <= j; ++i) H[(size_t)j * (m_max + 1) + i] = hp[i] + hp[512 + i];
            const double hn = std::sqrt(std::max(hp[1023], 0.0));
            H[(size_t)j * (m_max + 1) + j + 1] = hn;
            if (h_history) h_history[j] = hn;
            m = j + 1;
            h_last = hn;
            for (int i = 0; i <= j + 1; ++i) col[i] = H[(size_t)j * (m_max + 1) + i];
            for (int i = 0; i < j; ++i) {
                const double a = col[i], b = col[i + 1];
                col[i] = gc[i] * a + gs[i] * b;
                col[i + 1] = -gs[i] * a + gc[i] * b;
            }
            const double d = std::hypot(col[j], col[j + 1]);
            gc[j] = d > 0 ? col[j] / d : 1.0;
            gs[j] = d > 0 ? col[j + 1] / d : 0.0;
            gamma = -gs[j] * gamma;
            const double res = gc[j] != 0 ? std::fabs(gamma) / std::fabs(gc[j])
                                          : std::numeric_limits<double>::infinity();
            if (res_history) res_history[j] = res;
            const double test = stop_rule == MM_ARN_STOP_H ? hn : res;
            if (!(test > eps_arn) || !(hn > 0)) break;
            hp[0] = hn;
            MM_HIP(hipMemcpyAsync(hd.ptr, hp, sizeof(double), hipMemcpyHostToDevice, s));
            scale_copy(ctx, n, v.as<double>(), hd.as<double>(), W + (int64_t)(j + 1) * n, 1);
        }
        M->arn_m = m;
        M->H.assign((size_t)(m + 1) * m, 0.0);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i <= m; ++i)
                M->H[(size_t)j * (m + 1) + i] = H[(size_t)j * (m_max + 1) + i];
        std::vector<double> Hm((size_t)m * m);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) Hm[(size_t)j * m + i] = H[(size_t)j * (m_max + 1) + i];
        z_from_ritz(ctx, p, nz, M, W, m, Hm, k, eps_lambda, nullptr, false, v.as<double>(),
                    mbd->blk.ptr ? mbd->blk.as<double>() : nullptr);
        const int kk = M->k;
        if (info) {
            info->m = m;
            info->k = kk;
            info->h_last = h_last;
            info->setup_seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        }
    } catch (...) {
        delete M;
        throw;
    }
    *out = M;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_defl_build_pcg(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                       const mm_precond *mbd, const double *b, int32_t k,
                                       double eps_lambda, double tol, int32_t m_max,
                                       double *theta, double *x_out, mm_arnoldi_info *info,
                                       mm_precond **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    auto t_start = std::chrono::steady_clock::now();
    check_pair(p, nz);
    MM_CHECK(mbd && mbd->kind == 0 && mbd->n_obs == p->n_obs && mbd->nc == p->nc, MM_E_INVALID,
             "defl: needs an M_BD handle of the same pointing");
    MM_CHECK(b, MM_E_INVALID, "defl: null b");
    const int64_t n = p->n();
    MM_CHECK(m_max >= 1 && m_max <= 500 && m_max <= n, MM_E_INVALID,
             "defl: m_max in [1, min(500, n)]");
    MM_CHECK(eps_lambda > 0 || (k >= 1 && k <= 63 && k <= m_max), MM_E_INVALID,
             "defl: k in [1, 63] and <= m_max");
    hipStream_t s = ctx->stream;
    auto *M = new mm_precond();
    try {
        M->kind = 1;
        M->n_obs = p->n_obs;
        M->nc = p->nc;
        M->rcond_min = mbd->rcond_min;
        M->inv.alloc(sizeof(double) * packed_sym(p->nc) * p->n_obs);
        MM_HIP(hipMemcpyAsync(M->inv.ptr, mbd->inv.ptr, sizeof(double) * packed_sym(p->nc) * p->n_obs,
                              hipMemcpyDeviceToDevice, s));
        M->W.alloc(sizeof(double) * n * (m_max + 1));
        double *W = M->W.as<double>();
        // PCG with M_BD from x_0 = 0 (tol 0: it runs m_max iterations unless
        // the residual vanishes), keeping v_j = z_j / sqrt(rho_j) and the
        // coefficients alpha_j, beta_j
        PcgWork w;
        w.alloc(n, 1);
        DBuf xd, sq;
        xd.alloc(sizeof(double) * n);
        sq.alloc(sizeof(double));
        MM_HIP(hipMemsetAsync(xd.ptr, 0, sizeof(double) * n, s));
        pcg_init_scalars(ctx, 1, w.sd, 0.0);
        dot_cols(ctx, n, 1, b, b, w.sd.bn2);
        MM_HIP(hipMemcpyAsync(w.r.ptr, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        pcg_apply_M(ctx, mbd, w, w.r.as<double>(), w.z.as<double>());
        pcg_after_rz(ctx, 1, w.sd, w.part.as<double>(), w.n_part, 1);
        MM_HIP(hipMemcpyAsync(w.pv.ptr, w.z.ptr, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        double *hp = pinned(ctx, sizeof(double) * 8);
        auto read_scalars = [&]() {  // rho, alpha, beta, breakdown flag, ||r||^2, ||b||^2
            MM_HIP(hipMemcpyAsync(hp, w.sd.rho, sizeof(double), hipMemcpyDeviceToHost, s));
            MM_HIP(hipMemcpyAsync(hp + 1, w.sd.alpha, sizeof(double), hipMemcpyDeviceToHost, s));
            MM_HIP(hipMemcpyAsync(hp + 2, w.sd.beta, sizeof(double), hipMemcpyDeviceToHost, s));
            MM_HIP(hipMemcpyAsync(reinterpret_cast<int *>(hp + 3), w.sd.brk, sizeof(int),
                                  hipMemcpyDeviceToHost, s));
            MM_HIP(hipMemcpyAsync(hp + 5, w.sd.rn2, sizeof(double), hipMemcpyDeviceToHost, s));
            MM_HIP(hipMemcpyAsync(hp + 6, w.sd.bn2, sizeof(double), hipMemcpyDeviceToHost, s));
            MM_HIP(hipStreamSynchronize(s));
        };
        auto save_v = [&](int j, double rho) {
            hp[4] = std::sqrt(rho);
            MM_HIP(hipMemcpyAsync(sq.ptr, hp + 4, sizeof(double), hipMemcpyHostToDevice, s));
            scale_copy(ctx, n, w.z.as<double>(), sq.as<double>(), W + (int64_t)j * n, 1);
            MM_HIP(hipStreamSynchronize(s));
        };
        read_scalars();
        MM_CHECK(hp[0] > 0 && std::isfinite(hp[0]), MM_E_INVALID, "defl: zero start vector");
        save_v(0, hp[0]);
        std::vector<double> alpha, beta;
        int m = 1;
        for (int j = 0; j < m_max; ++j) {
            pcg_iteration(ctx, p, nz, mbd, w, xd.as<double>());
            read_scalars();
            MM_CHECK(!*reinterpret_cast<int *>(hp + 3), MM_E_BREAKDOWN, "defl: PCG breakdown");
            alpha.push_back(hp[1]);
            beta.push_back(hp[2]);
            if (j + 1 == m_max || !(hp[0] > 0) || hp[5] <= tol * tol * hp[6]) break;
            save_v(j + 1, hp[0]);
            m = j + 2;
        }
        // T_m: T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = -sqrt(beta_j)/alpha_j
        std::vector<double> T((size_t)m * m, 0.0);
        for (int j = 0; j < m; ++j) {
            T[(size_t)j * m + j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
            if (j + 1 < m)
                T[(size_t)j * m + j + 1] = T[(size_t)(j + 1) * m + j] =
                    -std::sqrt(beta[j]) / alpha[j];
        }
        if (x_out)
            MM_HIP(hipMemcpyAsync(x_out, xd.ptr, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        M->arn_m = m;
        M->H.assign((size_t)(m + 1) * m, 0.0);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) M->H[(size_t)j * (m + 1) + i] = T[(size_t)j * m + i];
        z_from_ritz(ctx, p, nz, M, W, m, T, k, eps_lambda, theta, true);
        if (info) {
            info->m = m;
            info->k = M->k;
            info->h_last = std::sqrt(beta[m - 1]) / alpha[m - 1];
            info->setup_seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        }
    } catch (...) {
        delete M;
        throw;
    }
    *out = M;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_defl_export(mm_ctx *ctx, const mm_precond *M, int32_t *k, double *Z,
                                    double *AZ, double *E) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(M && M->kind == 1, MM_E_INVALID, "defl_export: not an M_2l handle");
    const int64_t n = M->n();
    if (k) *k = M->k;
    if (Z) MM_HIP(hipMemcpyAsync(Z, M->Z.ptr, sizeof(double) * n * M->k, hipMemcpyDeviceToDevice, ctx->stream));
    if (AZ) MM_HIP(hipMemcpyAsync(AZ, M->AZ.ptr, sizeof(double) * n * M->k, hipMemcpyDeviceToDevice, ctx->stream));
    if (E) MM_HIP(hipMemcpyAsync(E, M->E.ptr, sizeof(double) * M->k * M->k, hipMemcpyDeviceToDevice, ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
    API_END
    return MM_OK;
}

extern "C" mm_status mm_defl_arnoldi_export(mm_ctx *ctx, const mm_precond *M, int32_t *m,
                                            double *W, double *H) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(M && M->kind == 1, MM_E_INVALID, "arnoldi_export: not an M_2l handle");
    const int64_t n = M->n();
    if (m) *m = M->arn_m;
    if (W && M->arn_m > 0)
        MM_HIP(hipMemcpyAsync(W, M->W.ptr, sizeof(double) * n * (M->arn_m + 1),
                              hipMemcpyDeviceToDevice, ctx->stream));
    if (H) std::memcpy(H, M->H.data(), sizeof(double) * M->H.size());
    MM_HIP(hipStreamSynchronize(ctx->stream));
    API_END
    return MM_OK;
}

extern "C" mm_status mm_precond_apply(mm_ctx *ctx, const mm_precond *M, int32_t nrhs,
                                      const double *v, double *out) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(M && v && out && v != out, MM_E_INVALID, "precond_apply: bad arguments");
    check_nrhs(nrhs);
    precond_apply_impl(ctx, M, nrhs, v, out, nullptr, 0);
    API_END
    return MM_OK;
}

extern "C" void mm_precond_destroy(mm_precond *M) { delete M; }

// ================================================================== solve

static mm_status block_cg(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                          const mm_precond *M, int R, const double *b, double *x, double tol,
                          int max_iter, int check, bool use_graph, double *history,
                          mm_solve_info *info);

extern "C" mm_status mm_solve(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                              const mm_precond *M, int32_t nrhs, const double *b, double *x,
                              double tol, int32_t max_iter, uint32_t flags, double *history,
                              mm_solve_info *info) {
    if (!ctx) return MM_E_INVALID;
    mm_status result = MM_OK;
    API_BEGIN(ctx)
    check_pair(p, nz);
    check_nrhs(nrhs);
    MM_CHECK(b && x && b != x, MM_E_INVALID, "solve: bad b/x");
    MM_CHECK(tol >= 0 && max_iter >= 0, MM_E_INVALID, "solve: bad tol/max_iter");
    MM_CHECK(!M || (M->n_obs == p->n_obs && M->nc == p->nc), MM_E_INVALID, "solve: preconditioner of another pointing");
    MM_CHECK(!((flags & MM_SOLVE_BLOCK) && (flags & MM_SOLVE_FLEXIBLE)), MM_E_INVALID,
             "solve: the flexible beta is for independent columns, not block CG");
    if (flags & MM_SOLVE_BLOCK) {
        MM_CHECK(nrhs >= 2, MM_E_INVALID, "solve: block CG needs nrhs >= 2");
        result = block_cg(ctx, p, nz, M, nrhs, b, x, tol, max_iter, std::max(1u, flags & 0xffu),
                          (flags & MM_SOLVE_GRAPH) != 0, history, info);
        return result;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = ctx->stream;
    const int64_t n = p->n();
    const int R = nrhs;
    PcgWork w;
    w.flexible = (flags & MM_SOLVE_FLEXIBLE) != 0;
    w.alloc(n, R);
    DBuf hist;
    hist.alloc(sizeof(double) * (size_t)(max_iter + 1) * R);
    w.sd.hist = hist.as<double>();
    w.sd.hist_len = max_iter + 1;
    pcg_init_scalars(ctx, R, w.sd, tol);
    dot_cols(ctx, n, R, b, b, w.sd.bn2);
    // r = b - A x0
    apply_A_impl(ctx, p, nz, R, x, w.q.as<double>());
    axpby_cols(ctx, n, R, b, w.q.as<double>(), w.r.as<double>());
    dot_partial_cols(ctx, n, R, w.r.as<double>(), w.r.as<double>(), w.part.as<double>(), w.n_part);
    pcg_after_rn(ctx, R, w.sd, w.part.as<double>(), w.n_part, 0);
    // z = M r, rho = r.z, p = z
    pcg_apply_M(ctx, M, w, w.r.as<double>(), w.z.as<double>());
    pcg_after_rz(ctx, R, w.sd, w.part.as<double>(), w.n_part, 1);
    MM_HIP(hipMemcpyAsync(w.pv.ptr, w.z.ptr, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
    std::vector<double> h_rn2((size_t)(max_iter + 1) * R, -1.0);
    int *hpin = reinterpret_cast<int *>(pinned(ctx, sizeof(int) * 64));
    const int check = std::max(1u, flags & 0xffu);
    const bool use_graph = (flags & MM_SOLVE_GRAPH) != 0;
    PcgGraph G;
    int it = 0;
    auto poll = [&]() -> bool {
        MM_HIP(hipMemcpyAsync(hpin, w.sd.done, sizeof(int) * R, hipMemcpyDeviceToHost, s));
        MM_HIP(hipStreamSynchronize(s));
        for (int c = 0; c < R; ++c)
            if (!hpin[c]) return false;
        return true;
    };
    bool all_done = poll();
    while (!all_done && it < max_iter) {
        if (use_graph && it >= 1 && it + check <= max_iter) {
            // first iteration ran eagerly (workspace sized); later chunks replay a graph
            G.drop_if_stale(ctx);
            if (!G.ex) capture_chunk(ctx, G, check, [&]() { pcg_iteration(ctx, p, nz, M, w, x); });
            MM_HIP(hipGraphLaunch(G.ex, s));
            it += check;
            all_done = poll();
            continue;
        }
        pcg_iteration(ctx, p, nz, M, w, x);
        ++it;
        if (it % check == 0 || it == max_iter || (use_graph && it == 1)) all_done = poll();
    }
    // true residual
    apply_A_impl(ctx, p, nz, R, x, w.q.as<double>());
    axpby_cols(ctx, n, R, b, w.q.as<double>(), w.r.as<double>());
    DBuf tr;
    tr.alloc(sizeof(double) * R);
    dot_cols(ctx, n, R, w.r.as<double>(), w.r.as<double>(), tr.as<double>());
    std::vector<double> h_tr(R), h_bn2(R), h_rn(R);
    std::vector<int> h_brk(R), h_it(R);
    MM_HIP(hipMemcpyAsync(h_tr.data(), tr.ptr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(h_bn2.data(), w.sd.bn2, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(h_rn.data(), w.sd.rn2, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(h_brk.data(), w.sd.brk, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(h_it.data(), w.sd.iters, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(h_rn2.data(), hist.ptr, sizeof(double) * (size_t)(it + 1) * R,
                          hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    std::vector<double> h_pr;
    if (info) precond_rel_res(ctx, M, n, R, w.r.as<double>(), b, w.z.as<double>(), h_pr);
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool any_brk = false, all_conv = true;
    for (int c = 0; c < R; ++c) {
        const double bn = h_bn2[c] > 0 ? std::sqrt(h_bn2[c]) : 1.0;
        const bool conv = !h_brk[c] && h_rn[c] <= tol * tol * h_bn2[c];
        any_brk |= h_brk[c] != 0;
        all_conv &= conv;
        if (info) {
            info[c].iters = h_it[c];
            info[c].converged = conv ? 1 : 0;
            info[c].breakdown = h_brk[c];
            info[c].pad = 0;
            info[c].rel_res_recursive = std::sqrt(std::max(h_rn[c], 0.0)) / bn;
            info[c].rel_res_true = std::sqrt(std::max(h_tr[c], 0.0)) / bn;
            info[c].solve_seconds = secs;
            info[c].rel_res_precond = h_pr[c];
        }
        if (history) {
            for (int k2 = 0; k2 <= max_iter; ++k2) {
                double v = -1.0;
                if (k2 <= h_it[c] && k2 <= it)
                    v = std::sqrt(std::max(h_rn2[(size_t)k2 * R + c], 0.0)) / bn;
                history[(size_t)c * (max_iter + 1) + k2] = v;
            }
        }
    }
    result = any_brk ? MM_E_BREAKDOWN : (all_conv ? MM_OK : MM_NOT_CONVERGED);
    if (any_brk) ctx->last_error = "PCG breakdown: p^T A p <= 0";
    API_END
    return result;
}

// ================================================ iterative refinement

extern "C" mm_status mm_solve_refined(mm_ctx *ctx, const mm_pointing *p_lo, const mm_noise *nz_lo,
                                      const mm_pointing *p_hi, const mm_noise *nz_hi,
                                      const mm_precond *M, int32_t nrhs, const double *b,
                                      double *x, double tol, double inner_tol, int32_t max_outer,
                                      int32_t max_inner, mm_refine_info *info) {
    if (!ctx) return MM_E_INVALID;
    mm_status result = MM_OK;
    API_BEGIN(ctx)
    const auto t0 = std::chrono::steady_clock::now();
    check_pair(p_lo, nz_lo);
    check_pair(p_hi, nz_hi);
    check_nrhs(nrhs);
    MM_CHECK(p_lo->n_samp == p_hi->n_samp && p_lo->n_obs == p_hi->n_obs && p_lo->nc == p_hi->nc,
             MM_E_INVALID, "refine: the two pointings differ in samples or observed pixels");
    MM_CHECK(b && x && b != x, MM_E_INVALID, "refine: bad b/x");
    MM_CHECK(tol > 0 && inner_tol > 0 && max_outer >= 1 && max_inner >= 1, MM_E_INVALID,
             "refine: tol, inner_tol > 0 and max_outer, max_inner >= 1");
    MM_CHECK(!M || (M->n_obs == p_hi->n_obs && M->nc == p_hi->nc), MM_E_INVALID,
             "refine: preconditioner of another pointing");
    hipStream_t s = ctx->stream;
    const int64_t n = p_hi->n();
    const int R = nrhs;
    DBuf r, e, Ax, nb;
    r.alloc(sizeof(double) * n * R);
    e.alloc(sizeof(double) * n * R);
    Ax.alloc(sizeof(double) * n * R);
    nb.alloc(sizeof(double) * 2 * R);
    std::vector<double> h(2 * R);
    dot_cols(ctx, n, R, b, b, nb.as<double>());
    std::vector<mm_solve_info> inner(R);
    int outer = 0, inner_total = 0;
    double worst = 0;
    bool conv = false;
    for (;;) {
        // r = A_hi x - b and its norm
        apply_A_impl(ctx, p_hi, nz_hi, R, x, Ax.as<double>());
        axpby_cols(ctx, n, R, Ax.as<double>(), b, r.as<double>());
        dot_cols(ctx, n, R, r.as<double>(), r.as<double>(), nb.as<double>() + R);
        MM_HIP(hipMemcpyAsync(h.data(), nb.ptr, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, s));
        MM_HIP(hipStreamSynchronize(s));
        conv = true;
        worst = 0;
        for (int c = 0; c < R; ++c) {
            const double rel = h[c] > 0 ? std::sqrt(std::max(h[R + c], 0.0) / h[c]) : 0.0;
            worst = std::max(worst, rel);
            conv &= rel <= tol;
        }
        if (conv || outer == max_outer) break;
        // correction: A_lo e = r to the accuracy the remaining gap needs
        // (tol / residual, halved; at least inner_tol, at most 0.5), then x -= e
        const double itol = std::min(0.5, std::max(inner_tol, 0.5 * tol / worst));
        MM_HIP(hipMemsetAsync(e.ptr, 0, sizeof(double) * n * R, s));
        const mm_status st = mm_solve(ctx, p_lo, nz_lo, M, R, r.as<double>(), e.as<double>(),
                                      itol, max_inner, 4u, nullptr, inner.data());
        if (st < 0) throw Error(st, std::string("refine: inner solve: ") + ctx->last_error);
        int it = 0;
        for (int c = 0; c < R; ++c) it = std::max(it, inner[c].iters);
        inner_total += it;
        axpby_cols(ctx, n, R, x, e.as<double>(), Ax.as<double>());  // x - e
        MM_HIP(hipMemcpyAsync(x, Ax.ptr, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
        ++outer;
    }
    if (info) {
        info->outer = outer;
        info->inner_iters = inner_total;
        info->converged = conv ? 1 : 0;
        info->pad = 0;
        info->rel_res_true = worst;
        info->solve_seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    result = conv ? MM_OK : MM_NOT_CONVERGED;
    API_END
    return result;
}

// ============================================================= block CG

// Block PCG (O'Leary 1980) with A-orthonormal search blocks:
//   R = B - A X; Z = M R; P~ = Z; Q~ = A P~; U = chol_drop(P~^T Q~)^-T;
//   P = P~ U; Q = Q~ U;  repeat: alpha = P^T R; X += P alpha; R -= Q alpha;
//   Z = M R; beta = Q^T Z; P~ = Z - P beta; Q~ = A P~; U; P = P~ U; Q = Q~ U.
// P^T A P = I on the kept directions, so alpha and beta need no solves; the
// Gram and block products run on FP64 MFMA.  Convergence is checked every
// `check` iterations on each column's ||r|| / ||b||.  With use_graph (and no
// history), the iterations after the first are replayed in chunks of `check`
// from a captured HIP graph; the convergence test follows each chunk, so a
// solve may run up to check - 1 iterations past the one that converged.
static mm_status block_cg(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                          const mm_precond *M, int R, const double *b, double *x, double tol,
                          int max_iter, int check, bool use_graph, double *history,
                          mm_solve_info *info) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = ctx->stream;
    const int64_t n = p->n();
    const size_t vb = sizeof(double) * n * R;
    DBuf Rr, Z, Pb, Q, Qt, sm, ib, rn, bn;
    Rr.alloc(vb); Z.alloc(vb); Pb.alloc(vb); Q.alloc(vb); Qt.alloc(vb);
    sm.alloc(sizeof(double) * 3 * 64 * 64);
    ib.alloc(sizeof(int) * 64);
    rn.alloc(sizeof(double) * 64);
    bn.alloc(sizeof(double) * 64);
    double *G = sm.as<double>(), *U = G + 4096, *AB = G + 8192;
    const double tau = 1e-10;
    auto precond = [&](const double *in, double *out) {
        if (M) precond_apply_impl(ctx, M, R, in, out, nullptr, 0);
        else MM_HIP(hipMemcpyAsync(out, in, vb, hipMemcpyDeviceToDevice, s));
    };
    // direction update from P~ (in Z): Q~ = A P~, U, P = P~ U, Q = Q~ U
    auto orthonormalise = [&]() {
        apply_A_impl(ctx, p, nz, R, Z.as<double>(), Qt.as<double>());
        gram_mfma(ctx, n, R, R, Z.as<double>(), R, 1, Qt.as<double>(), R, 1, G);
        chol_inv_drop(ctx, R, G, tau, U, ib.as<int>());
        gemm_rows_small(ctx, n, R, Z.as<double>(), U, 1.0, 0.0, Pb.as<double>());
        gemm_rows_small(ctx, n, R, Qt.as<double>(), U, 1.0, 0.0, Q.as<double>());
    };
    dot_cols(ctx, n, R, b, b, bn.as<double>());
    apply_A_impl(ctx, p, nz, R, x, Q.as<double>());
    axpby_cols(ctx, n, R, b, Q.as<double>(), Rr.as<double>());
    dot_cols(ctx, n, R, Rr.as<double>(), Rr.as<double>(), rn.as<double>());
    std::vector<double> h_bn(R), h_rn(R), hist_rn;
    MM_HIP(hipMemcpyAsync(h_bn.data(), bn.ptr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(h_rn.data(), rn.ptr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    auto all_conv = [&]() {
        for (int c = 0; c < R; ++c)
            if (!(h_rn[c] <= tol * tol * h_bn[c])) return false;
        return true;
    };
    hist_rn.insert(hist_rn.end(), h_rn.begin(), h_rn.end());
    int it = 0;
    bool conv = all_conv();
    if (!conv) {
        precond(Rr.as<double>(), Z.as<double>());
        orthonormalise();
    }
    // one whole iteration: X, R update, then the next A-orthonormal block
    auto iteration = [&]() {
        gram_mfma(ctx, n, R, R, Pb.as<double>(), R, 1, Rr.as<double>(), R, 1, AB);    // alpha
        gemm_rows_small(ctx, n, R, Pb.as<double>(), AB, 1.0, 1.0, x);
        gemm_rows_small(ctx, n, R, Q.as<double>(), AB, -1.0, 1.0, Rr.as<double>());
        precond(Rr.as<double>(), Z.as<double>());
        gram_mfma(ctx, n, R, R, Q.as<double>(), R, 1, Z.as<double>(), R, 1, AB);      // beta
        gemm_rows_small(ctx, n, R, Pb.as<double>(), AB, -1.0, 1.0, Z.as<double>());   // P~
        orthonormalise();
    };
    PcgGraph Gr;
    while (!conv && it < max_iter) {
        if (use_graph && !history && it >= 1 && it + check <= max_iter) {
            Gr.drop_if_stale(ctx);
            if (!Gr.ex) capture_chunk(ctx, Gr, check, iteration);
            MM_HIP(hipGraphLaunch(Gr.ex, s));
            it += check;
            dot_cols(ctx, n, R, Rr.as<double>(), Rr.as<double>(), rn.as<double>());
            MM_HIP(hipMemcpyAsync(h_rn.data(), rn.ptr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
            MM_HIP(hipStreamSynchronize(s));
            conv = all_conv();
            continue;
        }
        gram_mfma(ctx, n, R, R, Pb.as<double>(), R, 1, Rr.as<double>(), R, 1, AB);    // alpha
        gemm_rows_small(ctx, n, R, Pb.as<double>(), AB, 1.0, 1.0, x);
        gemm_rows_small(ctx, n, R, Q.as<double>(), AB, -1.0, 1.0, Rr.as<double>());
        ++it;
        const bool poll = (it % check == 0) || it == max_iter || history;
        if (poll) {
            dot_cols(ctx, n, R, Rr.as<double>(), Rr.as<double>(), rn.as<double>());
            MM_HIP(hipMemcpyAsync(h_rn.data(), rn.ptr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
            MM_HIP(hipStreamSynchronize(s));
            if (history) hist_rn.insert(hist_rn.end(), h_rn.begin(), h_rn.end());
            conv = all_conv();
            if (conv || it == max_iter) break;
        }
        precond(Rr.as<double>(), Z.as<double>());
        gram_mfma(ctx, n, R, R, Q.as<double>(), R, 1, Z.as<double>(), R, 1, AB);      // beta
        gemm_rows_small(ctx, n, R, Pb.as<double>(), AB, -1.0, 1.0, Z.as<double>());   // P~
        orthonormalise();
    }
    // true residuals
    apply_A_impl(ctx, p, nz, R, x, Q.as<double>());
    axpby_cols(ctx, n, R, b, Q.as<double>(), Rr.as<double>());
    dot_cols(ctx, n, R, Rr.as<double>(), Rr.as<double>(), rn.as<double>());
    std::vector<double> h_tr(R);
    MM_HIP(hipMemcpyAsync(h_tr.data(), rn.ptr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    std::vector<double> h_pr;
    if (info) precond_rel_res(ctx, M, n, R, Rr.as<double>(), b, Z.as<double>(), h_pr);
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    const int nh = (int)(hist_rn.size() / R);
    for (int c = 0; c < R; ++c) {
        const double bnc = h_bn[c] > 0 ? std::sqrt(h_bn[c]) : 1.0;
        const bool cv = h_rn[c] <= tol * tol * h_bn[c];
        all &= cv;
        if (info) {
            info[c].iters = it;
            info[c].converged = cv;
            info[c].breakdown = 0;
            info[c].pad = 0;
            info[c].rel_res_recursive = std::sqrt(std::max(h_rn[c], 0.0)) / bnc;
            info[c].rel_res_true = std::sqrt(std::max(h_tr[c], 0.0)) / bnc;
            info[c].solve_seconds = secs;
            info[c].rel_res_precond = h_pr[c];
        }
        if (history)
            for (int k2 = 0; k2 <= max_iter; ++k2)
                history[(size_t)c * (max_iter + 1) + k2] =
                    k2 < nh ? std::sqrt(std::max(hist_rn[(size_t)k2 * R + c], 0.0)) / bnc : -1.0;
    }
    return all ? MM_OK : MM_NOT_CONVERGED;
}

// ========================================================== PCG sessions

struct mm_pcg {
    const mm_pointing *p = nullptr;
    const mm_noise *nz = nullptr;
    const mm_precond *M = nullptr;
    PcgWork w;
    DBuf x, tb;
    int graph_chunk = 0;
    bool warm = false;
    PcgGraph G;
    std::vector<int> state, host_iters, max_iter;
    std::vector<double> tol;
};

extern "C" mm_status mm_pcg_create(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                   const mm_precond *M, int32_t nrhs, mm_pcg **out) {
    if (!ctx || !out) return MM_E_INVALID;
    *out = nullptr;
    API_BEGIN(ctx)
    check_pair(p, nz);
    check_nrhs(nrhs);
    MM_CHECK(!M || (M->n_obs == p->n_obs && M->nc == p->nc), MM_E_INVALID, "pcg: preconditioner of another pointing");
    auto *S = new mm_pcg();
    try {
        S->p = p;
        S->nz = nz;
        S->M = M;
        const int64_t n = p->n();
        S->w.alloc(n, nrhs);
        S->x.alloc(sizeof(double) * n * nrhs);
        S->tb.alloc(sizeof(double) * n);
        MM_HIP(hipMemsetAsync(S->x.ptr, 0, sizeof(double) * n * nrhs, ctx->stream));
        MM_HIP(hipMemsetAsync(S->w.r.ptr, 0, sizeof(double) * n * nrhs, ctx->stream));
        MM_HIP(hipMemsetAsync(S->w.pv.ptr, 0, sizeof(double) * n * nrhs, ctx->stream));
        pcg_init_scalars(ctx, nrhs, S->w.sd, 0.0);
        for (int c = 0; c < nrhs; ++c) slot_ctl(ctx, S->w.sd, c, 0, 0.0);
        S->state.assign(nrhs, 0);
        S->host_iters.assign(nrhs, 0);
        S->max_iter.assign(nrhs, 0);
        S->tol.assign(nrhs, 0.0);
        MM_HIP(hipStreamSynchronize(ctx->stream));
    } catch (...) {
        delete S;
        throw;
    }
    *out = S;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pcg_start(mm_ctx *ctx, mm_pcg *S, int32_t slot, const double *b,
                                  double tol, int32_t max_iter) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(S && b, MM_E_INVALID, "pcg_start: null argument");
    MM_CHECK(slot >= 0 && slot < S->w.R, MM_E_INVALID, "pcg_start: slot out of range");
    MM_CHECK(tol >= 0 && max_iter >= 0, MM_E_INVALID, "pcg_start: bad tol/max_iter");
    PcgWork &w = S->w;
    const int64_t n = w.n;
    double *z1 = S->tb.as<double>();
    // x = 0, r = b, z = M b, p = z
    col_set(ctx, n, w.R, slot, nullptr, S->x.as<double>());
    col_set(ctx, n, w.R, slot, b, w.r.as<double>());
    if (S->M)
        precond_apply_impl(ctx, S->M, 1, b, z1, nullptr, 0);
    else
        MM_HIP(hipMemcpyAsync(z1, b, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
    col_set(ctx, n, w.R, slot, z1, w.pv.as<double>());
    dot_cols(ctx, n, 1, b, b, w.sd.bn2 + slot);
    dot_cols(ctx, n, 1, b, z1, w.sd.rho + slot);
    slot_ctl(ctx, w.sd, slot, 1, tol);
    S->state[slot] = 1;
    S->host_iters[slot] = 0;
    S->max_iter[slot] = max_iter;
    S->tol[slot] = tol;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pcg_iterate(mm_ctx *ctx, mm_pcg *S, int32_t n_iter) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(S && n_iter >= 0, MM_E_INVALID, "pcg_iterate: bad arguments");
    int left = n_iter;
    while (left > 0) {
        int chunk = left;
        bool any = false;
        for (int c = 0; c < S->w.R; ++c)
            if (S->state[c] == 1) {
                const int rem = S->max_iter[c] - S->host_iters[c];
                if (rem <= 0) {
                    slot_ctl(ctx, S->w.sd, c, 0, 0.0);
                    S->state[c] = 5;  // budget spent; classified at the next poll
                    continue;
                }
                any = true;
                chunk = std::min(chunk, rem);
            }
        if (!any) break;
        int done_it = 0;
        if (S->graph_chunk > 0 && S->warm) {
            while (done_it + S->graph_chunk <= chunk) {
                S->G.drop_if_stale(ctx);
                if (!S->G.ex)
                    capture_chunk(ctx, S->G, S->graph_chunk, [&]() {
                        pcg_iteration(ctx, S->p, S->nz, S->M, S->w, S->x.as<double>());
                    });
                MM_HIP(hipGraphLaunch(S->G.ex, ctx->stream));
                done_it += S->graph_chunk;
            }
        }
        for (; done_it < chunk; ++done_it) {
            pcg_iteration(ctx, S->p, S->nz, S->M, S->w, S->x.as<double>());
            S->warm = true;
        }
        for (int c = 0; c < S->w.R; ++c)
            if (S->state[c] == 1) {
                S->host_iters[c] += chunk;
                if (S->host_iters[c] >= S->max_iter[c]) {
                    slot_ctl(ctx, S->w.sd, c, 0, 0.0);
                    S->state[c] = 5;
                }
            }
        left -= chunk;
    }
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pcg_use_graph(mm_ctx *ctx, mm_pcg *S, int32_t chunk) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(S && chunk >= 0 && chunk <= 1024, MM_E_INVALID, "pcg_use_graph: bad arguments");
    if (chunk != S->graph_chunk) {
        S->G.~PcgGraph();
        new (&S->G) PcgGraph();
        S->graph_chunk = chunk;
    }
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pcg_poll(mm_ctx *ctx, mm_pcg *S, int32_t *state, int32_t *iters,
                                 double *rel_res) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(S, MM_E_INVALID, "pcg_poll: null session");
    const int R = S->w.R;
    std::vector<int> dn(R), br(R), it(R);
    std::vector<double> rn(R), bn(R);
    hipStream_t s = ctx->stream;
    MM_HIP(hipMemcpyAsync(dn.data(), S->w.sd.done, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(br.data(), S->w.sd.brk, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(it.data(), S->w.sd.iters, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(rn.data(), S->w.sd.rn2, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(bn.data(), S->w.sd.bn2, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < R; ++c) {
        if (S->state[c] == 1 || S->state[c] == 5) {
            if (dn[c] || S->state[c] == 5) {
                const double t2 = S->tol[c] * S->tol[c];
                S->state[c] = br[c] ? 4 : (rn[c] <= t2 * bn[c] ? 2 : 3);
            }
        }
        if (state) state[c] = S->state[c];
        if (iters) iters[c] = S->state[c] == 0 ? 0 : it[c];
        if (rel_res)
            rel_res[c] = (S->state[c] == 0) ? 0.0
                         : std::sqrt(std::max(rn[c], 0.0)) / (bn[c] > 0 ? std::sqrt(bn[c]) : 1.0);
    }
    API_END
    return MM_OK;
}

extern "C" mm_status mm_pcg_finish(mm_ctx *ctx, mm_pcg *S, int32_t slot, double *x) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(S && x, MM_E_INVALID, "pcg_finish: null argument");
    MM_CHECK(slot >= 0 && slot < S->w.R, MM_E_INVALID, "pcg_finish: slot out of range");
    col_get(ctx, S->w.n, S->w.R, slot, S->x.as<double>(), x);
    slot_ctl(ctx, S->w.sd, slot, 0, 0.0);
    S->state[slot] = 0;
    MM_HIP(hipStreamSynchronize(ctx->stream));
    API_END
    return MM_OK;
}

extern "C" void mm_pcg_destroy(mm_pcg *S) { delete S; }

// ============================================================== autotune

extern "C" mm_status mm_autotune(mm_ctx *ctx, mm_pointing *p, mm_noise *nz, int32_t nrhs,
                                 int32_t flags, double *report, int32_t max_report,
                                 int32_t *n_report) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    check_pair(p, nz);
    check_nrhs(nrhs);
    MM_CHECK(max_report >= 0 && (report || max_report == 0), MM_E_INVALID,
             "autotune: report needs max_report entries");
    int nr = 0;
    autotune(ctx, p, nz, nrhs, flags, report, &nr, max_report);
    if (n_report) *n_report = nr;
    API_END
    return MM_OK;
}

// ======================================================= dense products

extern "C" mm_status mm_dense_gram(mm_ctx *ctx, int64_t n, int32_t ka, int32_t kb,
                                   const double *X, int64_t x_rs, int64_t x_cs, const double *Y,
                                   int64_t y_rs, int64_t y_cs, double *C) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(n >= 1 && ka >= 1 && ka <= 64 && kb >= 1 && kb <= 64 && X && Y && C, MM_E_INVALID,
             "dense_gram: sizes in [1, 64] and non-null arrays");
    gram_mfma(ctx, n, ka, kb, X, x_rs, x_cs, Y, y_rs, y_cs, C);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_dense_tall(mm_ctx *ctx, int64_t n, int32_t kin, int32_t kout,
                                   const double *V, const double *Y, double *Z) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(n >= 1 && kin >= 1 && kout >= 1 && kout <= 64 && V && Y && Z && Z != V, MM_E_INVALID,
             "dense_tall: kin >= 1, kout in [1, 64], distinct non-null arrays");
    matmul_small_right(ctx, n, kin, kout, V, Y, Z);
    API_END
    return MM_OK;
}

extern "C" mm_status mm_dense_rows(mm_ctx *ctx, int64_t n, int32_t R, const double *In,
                                   const double *S, double alpha, double beta, double *Out) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    check_nrhs(R);
    MM_CHECK(n >= 1 && In && S && Out && In != Out, MM_E_INVALID,
             "dense_rows: distinct non-null arrays");
    gemm_rows_small(ctx, n, R, In, S, alpha, beta, Out);
    API_END
    return MM_OK;
}

// ============================================================== profiling

extern "C" mm_status mm_profile_enable(mm_ctx *ctx, int on) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    ctx->prof.flush();
    ctx->prof.on = on != 0;
    API_END
    return MM_OK;
}

extern "C" mm_status mm_profile_read(mm_ctx *ctx, int32_t max, char *names, double *ms,
                                     int64_t *calls, int32_t *n) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    ctx->prof.flush();
    int i = 0;
    for (auto &kv : ctx->prof.stages) {
        if (i < max) {
            if (names) {
                std::memset(names + 32 * i, 0, 32);
                std::strncpy(names + 32 * i, kv.first.c_str(), 31);
            }
            if (ms) ms[i] = kv.second.ms;
            if (calls) calls[i] = kv.second.calls;
        }
        ++i;
    }
    if (n) *n = i;
    ctx->prof.stages.clear();
    API_END
    return MM_OK;
}

// =============================================================== host-only

extern "C" mm_status mm_hessenberg_eig(int32_t m, const double *H, double *wr, double *wi,
                                       double *vr, double *vi) {
    if (m < 1 || !H || !wr || !wi || !vr || !vi) return MM_E_INVALID;
    try {
        hessenberg_eig(m, H, wr, wi, vr, vi);
    } catch (const mm::Error &e) {
        return e.code;
    } catch (...) {
        return MM_E_DEVICE;
    }
    return MM_OK;
}
