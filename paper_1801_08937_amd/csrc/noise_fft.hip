// N^-1 by FFT: overlap-save convolution per stationary interval.
//
// For an interval [a, e) with half bandwidth lambda, the outputs
// t in [t0, t0 + V) need the inputs u in [t0 - lambda, t0 - lambda + N)
// (zero outside the interval), N = 2 NC real samples, V = N - 2 lambda.  A
// circular convolution of length N with the symmetric kernel
// h = (c_0, c_1 .. c_lambda, 0 .., c_lambda .. c_1) is then exact on those V
// outputs: no wrapped-around term reaches them.  The banded matrix is never
// formed; its spectrum H_k = c_0 + 2 sum_d c_d cos(2 pi k d / N) is real.
//
// One workgroup per block: the N real inputs are packed as NC complex values
// z_m = y_{2m} + i y_{2m+1}, transformed by an NC-point complex FFT held in
// LDS (Stockham, radices 16 x 8 x 8 x 8; the first forward pass reads global
// memory and the last inverse pass writes it, the others exchange through
// padded LDS), multiplied by the spectrum in the packed domain
//     Z'_k = A_k Z_k + B_k (W^k O_k + i W^-k E_k),
//     E_k = (Z_k + conj Z_{NC-k}) / 2,  O_k = (Z_k - conj Z_{NC-k}) / 2i,
//     A_k = (H_k + H_{k+NC}) / 2NC,     B_k = (H_k - H_{k+NC}) / 2NC,  W = e^{-2 pi i / N},
// and transformed back; the real and imaginary parts of the result are the
// even and odd outputs.
#include <algorithm>
#include <cmath>

#include "fft_common.h"

namespace mm {
namespace {

using fft::dft_small;

constexpr int FFT_NC = 8192;       // complex points per block
constexpr int FFT_N = 2 * FFT_NC;  // real samples per block
constexpr int FFT_THREADS = 512;

// LDS index with one pad slot per 16 entries, so the stride-16 accesses of
// the radix-16 pass fall in distinct banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
constexpr int FFT_LDS = FFT_NC + FFT_NC / 16;

// Twiddles e^{DIR 2 pi i jm r SCALE / NC} for r = 1..R-1 from one table entry
// (w1, r = 1) and products of at most three factors (w2 = w1^2, w4, w8).
template <typename T, int R, int DIR>
__device__ __forceinline__ void apply_twiddles(T (&re)[R], T (&im)[R], int jm, int scale,
                                               const typename Vec2T<T>::type *__restrict__ tw) {
    const auto t1 = tw[jm * scale];
    T wr[R], wi[R];
    wr[1] = t1.x;
    wi[1] = DIR < 0 ? t1.y : -t1.y;
#pragma unroll
    for (int r = 2; r < R; ++r) {
        // r = hi + lo with hi the largest power of two <= r (hi = r when r is a power of two)
        int hi = 1;
        while (hi * 2 <= r) hi *= 2;
        const int lo = r - hi;
        if (lo == 0) {
            const int h = hi / 2;
            wr[r] = wr[h] * wr[h] - wi[h] * wi[h];
            wi[r] = 2 * wr[h] * wi[h];
        } else {
            wr[r] = wr[hi] * wr[lo] - wi[hi] * wi[lo];
            wi[r] = wr[hi] * wi[lo] + wi[hi] * wr[lo];
        }
    }
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const T xr = re[r], xi = im[r];
        re[r] = wr[r] * xr - wi[r] * xi;
        im[r] = wr[r] * xi + wi[r] * xr;
    }
}

// A Stockham pass of radix R at sub-transform size NS, LDS to LDS:
// butterfly j reads x[j + r NC/R], twiddles by e^{DIR 2 pi i (j mod NS) r/(NS R)},
// and writes x[(j/NS) NS R + j mod NS + r NS].
template <typename T, int R, int NS, int DIR>
__device__ __forceinline__ void pass_lds(T *__restrict__ sre, T *__restrict__ sim,
                                         const typename Vec2T<T>::type *__restrict__ tw) {
    constexpr int NB = FFT_NC / R;
    constexpr int PER = NB / FFT_THREADS;
    T re[PER][R], im[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = tid + p * FFT_THREADS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            re[p][r] = sre[pad(j + r * NB)];
            im[p][r] = sim[pad(j + r * NB)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = tid + p * FFT_THREADS;
        const int jm = j % NS;
        if (NS > 1) apply_twiddles<T, R, DIR>(re[p], im[p], jm, FFT_NC / (NS * R), tw);
        dft_small<T, R, DIR>(re[p], im[p]);
        const int idx = (j / NS) * NS * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sre[pad(idx + r * NS)] = re[p][r];
            sim[pad(idx + r * NS)] = im[p][r];
        }
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(FFT_THREADS)
    k_noise_fft(const int64_t *__restrict__ blocks, const int64_t *__restrict__ istart,
                const int32_t *__restrict__ fid, const typename Vec2T<T>::type *__restrict__ ab,
                const typename Vec2T<T>::type *__restrict__ tw,
                const typename Vec2T<T>::type *__restrict__ twN, int lam, int V, int R,
                const T *__restrict__ y, T *__restrict__ z) {
    __shared__ T sre[FFT_LDS];
    __shared__ T sim[FFT_LDS];
    const int tid = threadIdx.x;
    const int rr = blockIdx.y;
    const int64_t t0 = blocks[2 * blockIdx.x];
    const int64_t iv = blocks[2 * blockIdx.x + 1];
    const int64_t a = istart[iv], e = istart[iv + 1];
    const int64_t base = t0 - lam;

    // forward pass 1 (radix 16, NS = 1) straight from global memory:
    // butterfly j takes z_m, m = j + 512 r, z_m = y_{base+2m} + i y_{base+2m+1}
    {
        T re[16], im[16];
        const int j = tid;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t u0 = base + 2 * (int64_t)(j + 512 * r), u1 = u0 + 1;
            re[r] = (u0 >= a && u0 < e) ? y[u0 * R + rr] : (T)0;
            im[r] = (u1 >= a && u1 < e) ? y[u1 * R + rr] : (T)0;
        }
        dft_small<T, 16, -1>(re, im);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            sre[pad(j * 16 + r)] = re[r];
            sim[pad(j * 16 + r)] = im[r];
        }
        __syncthreads();
    }
    pass_lds<T, 8, 16, -1>(sre, sim, tw);
    pass_lds<T, 8, 128, -1>(sre, sim, tw);
    pass_lds<T, 8, 1024, -1>(sre, sim, tw);

    // spectrum in the packed domain, one (k, NC-k) pair per thread step
    const auto *abf = ab + (int64_t)fid[iv] * FFT_NC;
    for (int k = tid; k <= FFT_NC / 2; k += FFT_THREADS) {
        const int kp = (FFT_NC - k) & (FFT_NC - 1);
        const T zr = sre[pad(k)], zi = sim[pad(k)], pr = sre[pad(kp)], pi = sim[pad(kp)];
        {
            const T er = (zr + pr) * (T)0.5, ei = (zi - pi) * (T)0.5;   // E = (Z + conj Zp)/2
            const T orr = (zi + pi) * (T)0.5, oi = -(zr - pr) * (T)0.5; // O = (Z - conj Zp)/2i
            const auto w = twN[k];
            const T wr = w.x, wi = w.y;                                 // W^k
            const T a1r = wr * orr - wi * oi, a1i = wr * oi + wi * orr; // W^k O
            const T b1r = wr * er + wi * ei, b1i = wr * ei - wi * er;   // W^-k E
            const T sr = a1r - b1i, si = a1i + b1r;                     // W^k O + i W^-k E
            const auto c = abf[k];
            sre[pad(k)] = c.x * zr + c.y * sr;
            sim[pad(k)] = c.x * zi + c.y * si;
        }
        if (kp != k) {
            const T er = (pr + zr) * (T)0.5, ei = (pi - zi) * (T)0.5;
            const T orr = (pi + zi) * (T)0.5, oi = -(pr - zr) * (T)0.5;
            const auto w = twN[kp];
            const T wr = w.x, wi = w.y;
            const T a1r = wr * orr - wi * oi, a1i = wr * oi + wi * orr;
            const T b1r = wr * er + wi * ei, b1i = wr * ei - wi * er;
            const T sr = a1r - b1i, si = a1i + b1r;
            const auto c = abf[kp];
            sre[pad(kp)] = c.x * pr + c.y * sr;
            sim[pad(kp)] = c.x * pi + c.y * si;
        }
    }
    __syncthreads();

    // inverse
    pass_lds<T, 16, 1, 1>(sre, sim, tw);
    pass_lds<T, 8, 16, 1>(sre, sim, tw);
    pass_lds<T, 8, 128, 1>(sre, sim, tw);
    // last pass (radix 8, NS = 1024) straight to global memory: butterfly j
    // produces z'_m, m = j + 1024 r, i.e. outputs 2m and 2m + 1 of the block
    int64_t nvalid = e - t0;
    if (nvalid > V) nvalid = V;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int j = tid + p * FFT_THREADS;
        T re[8], im[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            re[r] = sre[pad(j + 1024 * r)];
            im[r] = sim[pad(j + 1024 * r)];
        }
        apply_twiddles<T, 8, 1>(re, im, j, FFT_NC / (1024 * 8), tw);
        dft_small<T, 8, 1>(re, im);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t q0 = 2 * (int64_t)(j + 1024 * r) - lam;  // output offset from t0
            if (q0 >= 0 && q0 < nvalid) z[(t0 + q0) * R + rr] = re[r];
            if (q0 + 1 >= 0 && q0 + 1 < nvalid) z[(t0 + q0 + 1) * R + rr] = im[r];
        }
    }
}

// H_k = c_0 + 2 sum_d c_d cos(2 pi k d / N) for k in [0, N/2].  The cosine of
// 2 pi m / N comes from a quarter-period table in LDS (m reduced by integer
// arithmetic, k d mod N, then folded by symmetry), so every angle is exact.
constexpr int QMAX = 8192;  // N/4 for the largest block
__global__ void __launch_bounds__(256)
    k_fft_spectrum(const double *__restrict__ band, int lam, int N,
                   const double *__restrict__ qtab, double *__restrict__ H) {
    __shared__ double sc[QMAX + 1];
    const int Q = N / 4;
    for (int m = threadIdx.x; m <= Q; m += 256) sc[m] = qtab[m];
    __syncthreads();
    const int f = blockIdx.y;
    const double *c = band + (int64_t)f * (lam + 1);
    const int NC = N / 2;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k > NC) return;
    double s = 0;
    for (int d = 1; d <= lam; ++d) {
        int m = (int)(((int64_t)k * d) & (N - 1));
        if (m > NC) m = N - m;                       // cos(2 pi m/N) = cos(2 pi (N-m)/N)
        const double v = m > Q ? -sc[NC - m] : sc[m];  // cos(pi - x) = -cos x
        s += c[d] * v;
    }
    H[(int64_t)f * (NC + 1) + k] = c[0] + 2.0 * s;
}

template <typename T>
__global__ void k_fft_ab(const double *__restrict__ H, int n_filters, int NC,
                         typename Vec2T<T>::type *__restrict__ ab) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n_filters * NC) return;
    const int64_t f = e / NC;
    const int k = (int)(e % NC);
    const double hk = H[f * (NC + 1) + k];
    const double hc = H[f * (NC + 1) + (NC - k)];  // H_{k+NC} = H_{NC-k}
    typename Vec2T<T>::type v;
    v.x = (T)((hk + hc) / (2.0 * NC));
    v.y = (T)((hk - hc) / (2.0 * NC));
    ab[e] = v;
}

}  // namespace

bool noise_fft_big_supported(int half_bw);
int noise_fft_big_nc();
void noise_fft_big_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z);

bool noise_fft_supported(int half_bw, int64_t min_len) {
    (void)min_len;
    return half_bw >= 1 && noise_fft_big_supported(half_bw);
}

// Measured time model of one overlap-save apply with N-sample blocks.  The
// blocks run in waves of one per CU (a block fills a CU), and a block takes a
// fixed time (transforms and exchanges: 1 for 16,384 samples, 1.56 for
// 32,768) plus 1e-5 per input sample it reads (reads are clipped to the
// interval).  Fitted to FP64 applies of 2^20, 2^23 and 2^27 samples in
// 2^16-sample intervals, lambda 16 to 2,048, for the smallest loss from a
// wrong pick: each measured case gets the faster size or one within 5 %.
static double fft_time_model(const mm_noise *nz, int N, int n_cu) {
    const int64_t lam = nz->half_bw, V = N - 2 * lam;
    int64_t nb = 0;
    double rd = 0;
    for (int i = 0; i < nz->n_int; ++i) {
        const int64_t a = nz->h_istart[i], e = nz->h_istart[i + 1];
        for (int64_t t = a; t < e; t += V, ++nb)
            rd += (double)(std::min(e, t - lam + N) - std::max(a, t - lam));
    }
    if (nb == 0) return 0;
    const double fixed = N == 2 * FFT_NC ? 1.0 : 1.56;
    const int64_t waves = (nb + n_cu - 1) / n_cu;
    return (double)waves * (fixed + 1e-5 * rd / (double)nb);
}

// Block size: 16,384 real samples (lambda <= 2048) when the model above
// does not find 32,768 faster.  Small applies favour the small blocks (more
// blocks fill the CUs), large ones the large blocks (fewer exchanges per
// sample, and 7/8 valid at lambda = 2,048 against 3/4).
void noise_fft_prepare(mm_ctx *ctx, mm_noise *nz) {
    hipStream_t s = ctx->stream;
    const int lam = nz->half_bw;
    MM_CHECK(noise_fft_supported(lam, 0), MM_E_INVALID, "FFT: bandwidth unsupported");
    const int big_nc = noise_fft_big_nc();
    const bool small = lam <= 2048 && fft_time_model(nz, 2 * FFT_NC, ctx->n_cu) <=
                                          fft_time_model(nz, 2 * big_nc, ctx->n_cu);
    const int NC = small ? FFT_NC : big_nc;
    const int N = 2 * NC;
    nz->fft_n = N;
    nz->fft_valid = N - 2 * lam;
    const bool f32 = nz->prec == MM_F32;
    const size_t e2 = f32 ? sizeof(float2) : sizeof(double2);
    // twiddle tables (long double on the host, rounded once)
    std::vector<double> qtab(N / 4 + 1);
    std::vector<double> tw(2 * NC), twN(2 * NC);
    const long double pi2 = 6.283185307179586476925286766559L;
    for (int m = 0; m <= N / 4; ++m) qtab[m] = (double)cosl(pi2 * m / N);
    for (int m = 0; m < NC; ++m) {
        tw[2 * m] = (double)cosl(pi2 * m / NC);
        tw[2 * m + 1] = (double)-sinl(pi2 * m / NC);
        twN[2 * m] = (double)cosl(pi2 * m / N);
        twN[2 * m + 1] = (double)-sinl(pi2 * m / N);
    }
    nz->fft_tw.alloc(2 * e2 * NC);  // tw then twN
    if (f32) {
        std::vector<float> a(4 * (size_t)NC);
        for (int i = 0; i < 2 * NC; ++i) {
            a[i] = (float)tw[i];
            a[2 * NC + i] = (float)twN[i];
        }
        MM_HIP(hipMemcpyAsync(nz->fft_tw.ptr, a.data(), sizeof(float) * a.size(),
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipStreamSynchronize(s));
    } else {
        MM_HIP(hipMemcpyAsync(nz->fft_tw.ptr, tw.data(), sizeof(double) * tw.size(),
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipMemcpyAsync(nz->fft_tw.as<double>() + 2 * NC, twN.data(),
                              sizeof(double) * twN.size(), hipMemcpyHostToDevice, s));
        MM_HIP(hipStreamSynchronize(s));
    }
    // spectra
    DBuf dq, H;
    dq.alloc(sizeof(double) * qtab.size());
    H.alloc(sizeof(double) * (size_t)nz->n_filters * (NC + 1));
    MM_HIP(hipMemcpyAsync(dq.ptr, qtab.data(), sizeof(double) * qtab.size(), hipMemcpyHostToDevice,
                          s));
    dim3 g((NC + 1 + 255) / 256, nz->n_filters);
    k_fft_spectrum<<<g, 256, 0, s>>>(nz->band64.as<double>(), lam, N, dq.as<double>(),
                                     H.as<double>());
    nz->fft_spec.alloc(e2 * (size_t)nz->n_filters * NC);
    const int64_t tot = (int64_t)nz->n_filters * NC;
    if (f32)
        k_fft_ab<float><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
            H.as<double>(), nz->n_filters, NC, nz->fft_spec.as<float2>());
    else
        k_fft_ab<double><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
            H.as<double>(), nz->n_filters, NC, nz->fft_spec.as<double2>());
    MM_HIP(hipGetLastError());
    // block table
    std::vector<int64_t> blocks;
    for (int i = 0; i < nz->n_int; ++i)
        for (int64_t t = nz->h_istart[i]; t < nz->h_istart[i + 1]; t += nz->fft_valid) {
            blocks.push_back(t);
            blocks.push_back(i);
        }
    nz->n_fft_blocks = (int64_t)blocks.size() / 2;
    nz->fft_blocks.alloc(sizeof(int64_t) * blocks.size());
    MM_HIP(hipMemcpyAsync(nz->fft_blocks.ptr, blocks.data(), sizeof(int64_t) * blocks.size(),
                          hipMemcpyHostToDevice, s));
    MM_HIP(hipStreamSynchronize(s));
}

void noise_fft_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z) {
    if (nz->fft_n != FFT_N) {
        noise_fft_big_apply_dev(ctx, nz, nrhs, y, z);
        return;
    }
    Scope sc(ctx->prof, ctx->stream, "Ninv_fft");
    dim3 grid((unsigned)nz->n_fft_blocks, nrhs);
    if (nz->prec == MM_F32) {
        const float2 *tw = nz->fft_tw.as<float2>();
        k_noise_fft<float><<<grid, FFT_THREADS, 0, ctx->stream>>>(
            nz->fft_blocks.as<int64_t>(), nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
            nz->fft_spec.as<float2>(), tw, tw + FFT_NC, nz->half_bw, nz->fft_valid, nrhs,
            static_cast<const float *>(y), static_cast<float *>(z));
    } else {
        const double2 *tw = nz->fft_tw.as<double2>();
        k_noise_fft<double><<<grid, FFT_THREADS, 0, ctx->stream>>>(
            nz->fft_blocks.as<int64_t>(), nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
            nz->fft_spec.as<double2>(), tw, tw + FFT_NC, nz->half_bw, nz->fft_valid, nrhs,
            static_cast<const double *>(y), static_cast<double *>(z));
    }
    MM_HIP(hipGetLastError());
}


}  // namespace mm
