// Polynomial template filter as the time-domain weight (Sect. 2, Eqs. filt
// and filtnoise; Sect. 4: long modes filtered by low-order polynomials per
// subscan):
//     F = W - W B (B^T W B)^-1 B^T W,
// B block diagonal over subscans, each block the Legendre polynomials
// P_0..P_p of the subscan time mapped onto [-1, 1], and W = diag(w) with w_t
// the white-noise weight of the sample's interval times the flag mask.  Per
// subscan s with weighted samples,
//     c = G_s^-1 B_s^T W y,   G_s = B_s^T W B_s,   (F y)_t = w_t (y_t - B_t c).
// A subscan with at most p + 1 weighted samples is fitted exactly, so its
// output is 0 (the pseudo-inverse value).
//
// G_s^-1 is formed once per subscan at build time (FP64, Cholesky), so the
// apply reads y twice (the second pass from cache) and writes z: 16 bytes per
// sample and per column, like the direct band.  One wave per (subscan,
// column): the p + 1 weighted moments are reduced across the wave in a fixed
// order, the fit coefficients formed from G_s^-1 by every lane, and the
// residuals written; each column's arithmetic ignores the other columns.
#include <cmath>

#include "mm_internal.h"

namespace mm {
namespace {

constexpr int BS = 256;
constexpr int PF_MAX_ORDER = 7;

// P_0..P_NP-1 at u by the three-term recurrence.
template <typename T, int NP>
__device__ __forceinline__ void legendre(T u, T (&P)[NP]) {
    P[0] = (T)1;
    if (NP > 1) P[1] = u;
#pragma unroll
    for (int k = 1; k + 1 < NP; ++k)
        P[k + 1] = ((T)(2 * k + 1) * u * P[k] - (T)k * P[k - 1]) / (T)(k + 1);
}

template <typename T>
__device__ __forceinline__ T subscan_u(int64_t t, int64_t a, int64_t L) {
    return L > 1 ? (T)(-1.0 + 2.0 * (double)(t - a) / (double)(L - 1)) : (T)0;
}

__device__ __forceinline__ bool unflagged(const uint32_t *__restrict__ mask, int64_t t) {
    return (mask[t >> 5] >> (t & 31)) & 1u;
}

// mask bit t = 1 when sample t is kept (j_t >= 0)
__global__ void k_pf_mask(const int32_t *__restrict__ j, int64_t n, uint32_t *__restrict__ mask) {
    const int64_t wd = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (wd * 32 >= n) return;
    uint32_t m = 0;
    for (int b = 0; b < 32; ++b) {
        const int64_t t = wd * 32 + b;
        if (t < n && j[t] >= 0) m |= 1u << b;
    }
    mask[wd] = m;
}

// Per subscan: G = B^T W B (FP64) and its inverse, or zeros when at most
// p + 1 samples carry weight.  One wave per subscan.
template <int NP>
__global__ void __launch_bounds__(BS) k_pf_gram(const int64_t *__restrict__ sub,
                                                const double *__restrict__ omega, int64_t n_sub,
                                                const uint32_t *__restrict__ mask,
                                                double *__restrict__ ginv) {
    const int lane = threadIdx.x & 63;
    const int64_t s = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    if (s >= n_sub) return;
    const int64_t a = sub[s], b = sub[s + 1], L = b - a;
    const double om = omega[s];
    double g[NP * NP];
#pragma unroll
    for (int e = 0; e < NP * NP; ++e) g[e] = 0;
    int cnt = 0;
    for (int64_t t = a + lane; t < b; t += 64) {
        if (!unflagged(mask, t) || !(om > 0)) continue;
        double P[NP];
        legendre<double, NP>(subscan_u<double>(t, a, L), P);
        ++cnt;
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int l = 0; l < NP; ++l) g[k * NP + l] += om * P[k] * P[l];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        cnt += __shfl_xor(cnt, m);
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) g[e] += __shfl_xor(g[e], m);
    }
    if (lane != 0) return;
    double *out = ginv + s * NP * NP;
    bool ok = cnt > NP;
    // Cholesky G = R R^T (R lower), then G^-1 = R^-T R^-1
    double R[NP * NP];
#pragma unroll
    for (int e = 0; e < NP * NP; ++e) R[e] = 0;
    for (int c = 0; c < NP && ok; ++c) {
        for (int r = c; r < NP; ++r) {
            double v = 0.5 * (g[r * NP + c] + g[c * NP + r]);
            for (int q = 0; q < c; ++q) v -= R[r * NP + q] * R[c * NP + q];
            if (r == c) {
                if (!(v > 0)) {
                    ok = false;
                    break;
                }
                R[c * NP + c] = sqrt(v);
            } else {
                R[r * NP + c] = v / R[c * NP + c];
            }
        }
    }
    if (!ok) {
        for (int e = 0; e < NP * NP; ++e) out[e] = 0;
        return;
    }
    double Ri[NP * NP];  // R^-1, lower
#pragma unroll
    for (int e = 0; e < NP * NP; ++e) Ri[e] = 0;
    for (int c = 0; c < NP; ++c) {
        Ri[c * NP + c] = 1.0 / R[c * NP + c];
        for (int r = c + 1; r < NP; ++r) {
            double v = 0;
            for (int q = c; q < r; ++q) v -= R[r * NP + q] * Ri[q * NP + c];
            Ri[r * NP + c] = v / R[r * NP + r];
        }
    }
    for (int k = 0; k < NP; ++k)
        for (int l = 0; l < NP; ++l) {
            double v = 0;
            for (int q = (k > l ? k : l); q < NP; ++q) v += Ri[q * NP + k] * Ri[q * NP + l];
            out[k * NP + l] = v;
        }
}

// z = F y for one (subscan, column) per wave.
template <typename T, int NP>
__global__ void __launch_bounds__(BS) k_pf_apply(const int64_t *__restrict__ sub,
                                                 const double *__restrict__ omega, int64_t n_sub,
                                                 const uint32_t *__restrict__ mask,
                                                 const double *__restrict__ ginv, int R,
                                                 const T *__restrict__ y, T *__restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int64_t s = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    if (s >= n_sub) return;
    const int r = blockIdx.y;
    const int64_t a = sub[s], b = sub[s + 1], L = b - a;
    const double *gi = ginv + s * NP * NP;
    const T om = (T)omega[s];
    bool live = false;
#pragma unroll
    for (int e = 0; e < NP; ++e) live |= gi[e * NP + e] != 0.0;
    if (!live) {
        for (int64_t t = a + lane; t < b; t += 64) z[t * R + r] = (T)0;
        return;
    }
    T mom[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) mom[k] = 0;
    for (int64_t t = a + lane; t < b; t += 64) {
        const T w = unflagged(mask, t) ? om : (T)0;
        const T wy = w * y[t * R + r];
        T P[NP];
        legendre<T, NP>(subscan_u<T>(t, a, L), P);
#pragma unroll
        for (int k = 0; k < NP; ++k) mom[k] += P[k] * wy;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
        for (int k = 0; k < NP; ++k) mom[k] += __shfl_xor(mom[k], m);
    T c[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        T v = 0;
#pragma unroll
        for (int l = 0; l < NP; ++l) v += (T)gi[k * NP + l] * mom[l];
        c[k] = v;
    }
    for (int64_t t = a + lane; t < b; t += 64) {
        const T w = unflagged(mask, t) ? om : (T)0;
        T P[NP];
        legendre<T, NP>(subscan_u<T>(t, a, L), P);
        T fit = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) fit += P[k] * c[k];
        z[t * R + r] = w * (y[t * R + r] - fit);
    }
}

template <typename F>
void dispatch_np(int np, F &&f) {
    switch (np) {
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        case 3: f(std::integral_constant<int, 3>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        case 5: f(std::integral_constant<int, 5>()); break;
        case 6: f(std::integral_constant<int, 6>()); break;
        case 7: f(std::integral_constant<int, 7>()); break;
        case 8: f(std::integral_constant<int, 8>()); break;
        default: throw Error(MM_E_INVALID, "polynomial order must be in [0, 7]");
    }
}

}  // namespace

int polyfilter_max_order() { return PF_MAX_ORDER; }

void polyfilter_prepare(mm_ctx *ctx, const mm_pointing *p, mm_noise *nz) {
    hipStream_t s = ctx->stream;
    const int64_t n = nz->n_samp;
    const int64_t nw = (n + 31) / 32;
    nz->pf_mask.alloc(sizeof(uint32_t) * nw);
    k_pf_mask<<<(unsigned)((nw + BS - 1) / BS), BS, 0, s>>>(p->j.as<int32_t>(), n,
                                                            nz->pf_mask.as<uint32_t>());
    const int NP = nz->pf_order + 1;
    nz->pf_ginv.alloc(sizeof(double) * (size_t)nz->pf_n_sub * NP * NP);
    const unsigned nb = (unsigned)((nz->pf_n_sub * 64 + BS - 1) / BS);
    dispatch_np(NP, [&](auto NN) {
        k_pf_gram<decltype(NN)::value><<<nb, BS, 0, s>>>(
            nz->pf_sub.as<int64_t>(), nz->pf_omega.as<double>(), nz->pf_n_sub,
            nz->pf_mask.as<uint32_t>(), nz->pf_ginv.as<double>());
    });
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(s));
}

void polyfilter_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z) {
    Scope sc(ctx->prof, ctx->stream, "Ninv_poly");
    const int NP = nz->pf_order + 1;
    dim3 grid((unsigned)((nz->pf_n_sub * 64 + BS - 1) / BS), nrhs);
    dispatch_np(NP, [&](auto NN) {
        constexpr int N = decltype(NN)::value;
        if (nz->prec == MM_F32)
            k_pf_apply<float, N><<<grid, BS, 0, ctx->stream>>>(
                nz->pf_sub.as<int64_t>(), nz->pf_omega.as<double>(), nz->pf_n_sub,
                nz->pf_mask.as<uint32_t>(), nz->pf_ginv.as<double>(), nrhs,
                static_cast<const float *>(y), static_cast<float *>(z));
        else
            k_pf_apply<double, N><<<grid, BS, 0, ctx->stream>>>(
                nz->pf_sub.as<int64_t>(), nz->pf_omega.as<double>(), nz->pf_n_sub,
                nz->pf_mask.as<uint32_t>(), nz->pf_ginv.as<double>(), nrhs,
                static_cast<const double *>(y), static_cast<double *>(z));
    });
    MM_HIP(hipGetLastError());
}

}  // namespace mm
