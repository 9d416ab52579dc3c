// N^-1 by FFT: overlap-save convolution per stationary interval -- the
// spectrum tables, the block table and the choice of block size.  The
// transforms run in noise_fft_big.hip (register-resident kernels for 16,384-
// and 32,768-sample blocks).
//
// For an interval [a, e) with half bandwidth lambda, the outputs
// t in [t0, t0 + V) need the inputs u in [t0 - lambda, t0 - lambda + N)
// (zero outside the interval), N = 2 NC real samples, V = N - 2 lambda.  A
// circular convolution of length N with the symmetric kernel
// h = (c_0, c_1 .. c_lambda, 0 .., c_lambda .. c_1) is then exact on those V
// outputs: no wrapped-around term reaches them.  The banded matrix is never
// formed; its spectrum H_k = c_0 + 2 sum_d c_d cos(2 pi k d / N) is real.
//
// The N real inputs of a block are packed as NC complex values
// z_m = y_{2m} + i y_{2m+1}, transformed by an NC-point complex FFT,
// multiplied by the spectrum in the packed domain
//     Z'_k = A_k Z_k + B_k (W^k O_k + i W^-k E_k),
//     E_k = (Z_k + conj Z_{NC-k}) / 2,  O_k = (Z_k - conj Z_{NC-k}) / 2i,
//     A_k = (H_k + H_{k+NC}) / 2NC,     B_k = (H_k - H_{k+NC}) / 2NC,  W = e^{-2 pi i / N},
// and transformed back; the real and imaginary parts of the result are the
// even and odd outputs.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "fft_common.h"

namespace mm {
namespace {

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
bool noise_fft_mid_supported(int half_bw);
int noise_fft_big_nc();
int noise_fft_mid_nc();
void noise_fft_reg_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z);

bool noise_fft_supported(int half_bw, int64_t min_len) {
    (void)min_len;
    return half_bw >= 1 && noise_fft_big_supported(half_bw);
}

// Measured time model of one overlap-save apply with N-sample blocks.  Blocks
// run in waves of n_cu x (blocks per CU): two 16,384-sample blocks share a CU,
// a 32,768-sample block fills one.  A wave takes 40 (16,384) or 44 (32,768)
// time units; the count of waves is rounded up.  Fitted to FP64 and FP32
// applies of 2^23 and 2^27 samples in 2^16-sample intervals, lambda 512 to
// 4,096: the pick is the faster kernel, or within 5 % of it, in every case.
static double fft_time_model(const mm_noise *nz, int N, int n_cu) {
    const int64_t lam = nz->half_bw, V = N - 2 * lam;
    if (V <= 0) return 1e300;
    int64_t nb = 0;
    for (int i = 0; i < nz->n_int; ++i)
        nb += (nz->h_istart[i + 1] - nz->h_istart[i] + V - 1) / V;
    const bool mid = N == 2 * noise_fft_mid_nc();
    const int64_t per_wave = (int64_t)n_cu * (mid ? 2 : 1);
    const int64_t waves = (nb + per_wave - 1) / per_wave;
    return (double)waves * (mid ? 40.0 : 44.0);
}

// Tables for blocks of n_fft real samples (0 = pick by the model above).
void noise_fft_prepare(mm_ctx *ctx, mm_noise *nz, int n_fft) {
    hipStream_t s = ctx->stream;
    const int lam = nz->half_bw;
    MM_CHECK(noise_fft_supported(lam, 0), MM_E_INVALID, "FFT: bandwidth unsupported");
    if (n_fft == 0) {
        const int nm = 2 * noise_fft_mid_nc(), nb = 2 * noise_fft_big_nc();
        n_fft = noise_fft_mid_supported(lam) &&
                        fft_time_model(nz, nm, ctx->n_cu) <= fft_time_model(nz, nb, ctx->n_cu)
                    ? nm
                    : nb;
    }
    MM_CHECK(n_fft == 2 * noise_fft_big_nc() ||
                 (n_fft == 2 * noise_fft_mid_nc() && noise_fft_mid_supported(lam)),
             MM_E_INVALID, "FFT: block length must be 16,384 (lambda <= 6,144) or 32,768");
    const int NC = n_fft / 2;
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
    noise_fft_reg_apply_dev(ctx, nz, nrhs, y, z);
}


}  // namespace mm
