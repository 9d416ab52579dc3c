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
//
// Ground templates (Sect. 4, ground pickup): G[t, b] = 1 when sample t falls
// in azimuth bin b.  G^T W G is diagonal, so F_G y = W (y - G g) with g_b the
// w-weighted mean of bin b's samples (0 for a bin without weight).  With
// both template sets the filter is the symmetric combination
//     F = F_B W^+ F_G W^+ F_B = W (I - Pi_B)(I - Pi_G)(I - Pi_B),
// Pi_X = X (X^T W X)^+ X^T W, W^+ the pseudo-inverse (zero on flagged
// samples).  Apply: y1 = (I - Pi_B) y on weighted samples (0 elsewhere); per
// bin the weighted sums of y1 over fixed chunks of the bin's time-sorted
// samples, then g = (chunk sums in chunk order) / (sum of w); z = W (I - Pi_B)
// (y1 - G g), the subtraction done as the last pass reads y1.  No atomics:
// every sum has a fixed order.
#include <cmath>
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "mm_internal.h"

namespace mm {
namespace {

constexpr int BS = 256;
constexpr int PF_MAX_ORDER = 7;
constexpr int64_t GB_CHUNK = 512;  // entries per lane and wave of the ground sums

// P_0..P_NP-1 at u by the three-term recurrence.
template <typename T, int NP>
__device__ __forceinline__ void legendre(T u, T (&P)[NP]) {
    P[0] = (T)1;
    if constexpr (NP > 1) P[1] = u;
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

// Input value of sample t: y, minus its bin's ground amplitude when ghat is
// given.
template <typename T>
__device__ __forceinline__ T pf_value(const T *__restrict__ y, const int32_t *__restrict__ gbin,
                                      const T *__restrict__ ghat, int64_t t, int R, int r) {
    T v = y[t * R + r];
    if (ghat) {
        const int32_t g = gbin[t];
        if (g >= 0) v -= ghat[(int64_t)g * R + r];
    }
    return v;
}

// The apply for a subscan of at most 64 NV samples (the usual case): a
// lane's NV samples are loaded at once (clamped to the subscan, with no
// branch per sample), kept in registers for the second pass, and summed in
// the same order as the streaming loop of k_pf_apply, so the result is the
// same bits in one round trip instead of two per 64 samples.  NV is the
// smallest of 4 and 8 that holds the longest subscan: loads beyond it would
// be wasted issue slots and registers (measured: 0.51 against 0.67 ms for 4
// and 8 at 256-sample subscans).
template <typename T, int NP, int NV>
__device__ __forceinline__ void pf_apply_cached(int64_t a, int64_t b, int64_t L, int lane,
                                                const double *__restrict__ gi, T om,
                                                const uint32_t *__restrict__ mask, int R, int r,
                                                const T *__restrict__ y,
                                                const int32_t *__restrict__ gbin,
                                                const T *__restrict__ ghat, bool weighted,
                                                T *__restrict__ z) {
    T mom[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) mom[k] = 0;
    T val[NV];
    bool in[NV], on[NV];
    int64_t tc[NV];
    uint32_t mw[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int64_t t = a + lane + 64 * q;
        in[q] = t < b;
        tc[q] = in[q] ? t : a;
        val[q] = y[tc[q] * R + r];
        mw[q] = mask[tc[q] >> 5];
    }
    if (ghat) {  // bins, then their amplitudes, each batch in flight together
        int32_t g[NV];
        T gv[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) g[q] = gbin[tc[q]];
#pragma unroll
        for (int q = 0; q < NV; ++q) gv[q] = ghat[(int64_t)(g[q] < 0 ? 0 : g[q]) * R + r];
#pragma unroll
        for (int q = 0; q < NV; ++q) val[q] = g[q] >= 0 ? val[q] - gv[q] : val[q];
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) on[q] = in[q] && ((mw[q] >> (tc[q] & 31)) & 1u);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int64_t t = a + lane + 64 * q;
        const T wy = (on[q] ? om : (T)0) * val[q];
        T P[NP];
        legendre<T, NP>(subscan_u<T>(t, a, L), P);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const T nm = mom[k] + P[k] * wy;
            mom[k] = in[q] ? nm : mom[k];
        }
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
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (!in[q]) continue;
        const int64_t t = a + lane + 64 * q;
        const T w = on[q] ? om : (T)0;
        T P[NP];
        legendre<T, NP>(subscan_u<T>(t, a, L), P);
        T fit = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) fit += P[k] * c[k];
        const T res = val[q] - fit;
        z[t * R + r] = weighted ? w * res : (on[q] && om > (T)0 ? res : (T)0);
    }
}

// One (subscan, column) per wave: weighted ? z = W (v - B c) : z = v - B c on
// weighted samples and 0 elsewhere, with v the input value above and c the
// subscan's weighted fit to v.
template <typename T, int NP, int NV>
__global__ void __launch_bounds__(BS) k_pf_apply(const int64_t *__restrict__ sub,
                                                 const double *__restrict__ omega, int64_t n_sub,
                                                 const uint32_t *__restrict__ mask,
                                                 const double *__restrict__ ginv, int R,
                                                 const T *__restrict__ y,
                                                 const int32_t *__restrict__ gbin,
                                                 const T *__restrict__ ghat, bool weighted,
                                                 T *__restrict__ z) {
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
    if (L <= 0) return;  // no sample (the cached path clamps to the first one)
    if constexpr (NV > 0) {
        if (L <= 64 * NV) {
            pf_apply_cached<T, NP, NV>(a, b, L, lane, gi, om, mask, R, r, y, gbin, ghat, weighted,
                                       z);
            return;
        }
    }
    for (int64_t t = a + lane; t < b; t += 64) {
        const T w = unflagged(mask, t) ? om : (T)0;
        const T wy = w * pf_value(y, gbin, ghat, t, R, r);
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
        const bool on = unflagged(mask, t);
        const T w = on ? om : (T)0;
        T P[NP];
        legendre<T, NP>(subscan_u<T>(t, a, L), P);
        T fit = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) fit += P[k] * c[k];
        const T res = pf_value(y, gbin, ghat, t, R, r) - fit;
        z[t * R + r] = weighted ? w * res : (on && om > (T)0 ? res : (T)0);
    }
}

// --- ground templates -------------------------------------------------------

// bad[0] = 1 if a bin lies outside [-1, nb)
__global__ void k_gb_check(const int32_t *__restrict__ gbin, int64_t n, int32_t nb,
                           int *__restrict__ bad) {
    int b = 0;
    for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * BS) {
        const int32_t g = gbin[t];
        b |= g < -1 || g >= nb;
    }
    if (b) atomicOr(bad, 1);
}

// Sort keys (bin, samples without a bin last) and per-bin sample counts.
__global__ void k_gb_keys(const int32_t *__restrict__ gbin, int64_t n, int32_t nb,
                          uint32_t *__restrict__ key, int32_t *__restrict__ val,
                          int32_t *__restrict__ cnt) {
    for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * BS) {
        const int32_t g = gbin[t];
        key[t] = g >= 0 ? (uint32_t)g : (uint32_t)nb;
        val[t] = (int32_t)t;
        if (g >= 0) atomicAdd(cnt + g, 1);
    }
}

// w of each bin entry: the weight of the sample's subscan times its mask.
__global__ void k_gb_weights(const int32_t *__restrict__ gperm, int64_t nv,
                             const int64_t *__restrict__ sub, int64_t n_sub,
                             const double *__restrict__ omega, const uint32_t *__restrict__ mask,
                             double *__restrict__ gw) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * BS) {
        const int64_t t = gperm[i];
        int64_t lo = 0, hi = n_sub;  // last subscan with start <= t
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (sub[mid] <= t)
                lo = mid;
            else
                hi = mid;
        }
        gw[i] = unflagged(mask, t) ? omega[lo] : 0.0;
    }
}

// Interleaved bin layout.  Bins are taken 64 at a time (group g: bins 64 g
// + lane), and each group's entries are cut into chunks of at most GB_CHUNK
// per lane; wave w = one (group, chunk).  Entry i of lane l of wave w sits at
// base[w] + 64 i + l (padded with t = -1), so the 64 lanes read their bins'
// i-th samples together: for neighbouring azimuth bins those are neighbouring
// samples of one sweep, and the gather of y1 is coalesced.  Each lane sums
// its entries in order; the partial sums of a bin are added in chunk order.
template <typename T>
__global__ void __launch_bounds__(BS) k_gb_part(const int64_t *__restrict__ base,
                                                int32_t n_wave, const int32_t *__restrict__ sp,
                                                const double *__restrict__ sw, int R,
                                                const T *__restrict__ y1, T *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    if (w >= n_wave) return;
    const int r = blockIdx.y;
    const int64_t b0 = base[w];
    const int64_t W = (base[w + 1] - b0) >> 6;
    const int32_t *pp = sp + b0 + lane;
    const double *wp = sw + b0 + lane;
    T acc = 0;
    int64_t i = 0;
    // eight entries in flight: their samples and weights together, then the
    // eight gathers (a padding entry, -1, reads sample 0 and adds 0, so no
    // gather waits behind a branch), summed in entry order
    for (; i + 7 < W; i += 8) {
        int32_t t[8];
        double wv[8];
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            t[q] = pp[64 * (i + q)];
            wv[q] = wp[64 * (i + q)];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const T g = y1[(int64_t)(t[q] < 0 ? 0 : t[q]) * R + r];
            v[q] = t[q] >= 0 ? g : (T)0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += (T)wv[q] * v[q];
    }
    for (; i < W; ++i) {
        const int32_t t = pp[64 * i];
        if (t >= 0) acc += (T)wp[64 * i] * y1[(int64_t)t * R + r];
    }
    part[(w * R + r) * 64 + lane] = acc;
}

// ghat[b R + r] = (bin b's partial sums in chunk order) / (sum of w).
template <typename T>
__global__ void k_gb_final(const int32_t *__restrict__ first, int32_t nb,
                           const double *__restrict__ gwinv, int R, const T *__restrict__ part,
                           T *__restrict__ ghat) {
    const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (e >= (int64_t)nb * R) return;
    const int64_t b = e / R;
    const int r = (int)(e % R);
    const int64_t g = b >> 6, l = b & 63;
    T acc = 0;
    for (int64_t w = first[g]; w < first[g + 1]; ++w) acc += part[(w * R + r) * 64 + l];
    ghat[e] = acc * (T)gwinv[b];
}

// Fill the interleaved layout from the bin-sorted entries.
__global__ void k_gb_fill(const int64_t *__restrict__ base, int32_t n_wave,
                          const int32_t *__restrict__ wgroup, const int32_t *__restrict__ first,
                          const int64_t *__restrict__ goff, int32_t nb,
                          const int32_t *__restrict__ gperm, const double *__restrict__ gw,
                          int32_t *__restrict__ sp, double *__restrict__ sw) {
    const int lane = threadIdx.x & 63;
    const int64_t nwv = ((int64_t)gridDim.x * BS) >> 6;
    for (int64_t w = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6; w < n_wave; w += nwv) {
        const int32_t g = wgroup[w];
        const int64_t k = w - first[g];
        const int64_t b = (int64_t)g * 64 + lane;
        int64_t lo = 0, hi = 0;
        if (b < nb) {
            lo = goff[b] + k * GB_CHUNK;
            hi = goff[b + 1] < lo + GB_CHUNK ? goff[b + 1] : lo + GB_CHUNK;
        }
        const int64_t b0 = base[w];
        const int64_t W = (base[w + 1] - b0) >> 6;
        for (int64_t i = 0; i < W; ++i) {
            const int64_t src = lo + i;
            const int64_t dst = b0 + 64 * i + lane;
            const bool ok = src < hi;
            sp[dst] = ok ? gperm[src] : -1;
            sw[dst] = ok ? gw[src] : 0.0;
        }
    }
}

// 1 / (sum of w over bin b), 0 for a bin without weight; one wave per bin.
__global__ void __launch_bounds__(BS) k_gb_winv(const int64_t *__restrict__ goff, int32_t nb,
                                                const double *__restrict__ gw,
                                                double *__restrict__ gwinv) {
    const int lane = threadIdx.x & 63;
    const int64_t b = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    if (b >= nb) return;
    double acc = 0;
    for (int64_t i = goff[b] + lane; i < goff[b + 1]; i += 64) acc += gw[i];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    if (lane == 0) gwinv[b] = acc > 0 ? 1.0 / acc : 0.0;
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

int grid_for(int64_t n, int max_blocks = 8192) {
    int64_t g = (n + BS - 1) / BS;
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

// Bin table of the ground templates: samples sorted by (bin, time), each
// entry's weight, per-bin 1 / sum w, and chunks of at most GB_CHUNK entries
// that never cross a bin.
void ground_prepare(mm_ctx *ctx, mm_noise *nz, const int32_t *gbin, int32_t nb) {
    hipStream_t s = ctx->stream;
    const int64_t n = nz->n_samp;
    DBuf bad;
    bad.alloc(sizeof(int));
    MM_HIP(hipMemsetAsync(bad.ptr, 0, sizeof(int), s));
    k_gb_check<<<grid_for(n), BS, 0, s>>>(gbin, n, nb, bad.as<int>());
    int hb = 0;
    MM_HIP(hipMemcpyAsync(&hb, bad.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    MM_CHECK(!hb, MM_E_INVALID, "polyfilter: ground bin outside [-1, n_ground_bins)");

    DBuf key, val, key_o, cnt, tmp;
    key.alloc(sizeof(uint32_t) * n);
    val.alloc(sizeof(int32_t) * n);
    key_o.alloc(sizeof(uint32_t) * n);
    cnt.alloc(sizeof(int32_t) * nb);
    DBuf gperm;
    gperm.alloc(sizeof(int32_t) * n);
    nz->pf_gbin.alloc(sizeof(int32_t) * n);
    MM_HIP(hipMemcpyAsync(nz->pf_gbin.ptr, gbin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    MM_HIP(hipMemsetAsync(cnt.ptr, 0, sizeof(int32_t) * nb, s));
    k_gb_keys<<<grid_for(n), BS, 0, s>>>(gbin, n, nb, key.as<uint32_t>(), val.as<int32_t>(),
                                         cnt.as<int32_t>());
    unsigned end_bit = 1;
    while (end_bit < 32 && ((uint64_t)1 << end_bit) <= (uint64_t)nb) ++end_bit;
    size_t tb = 0;
    MM_HIP(rocprim::radix_sort_pairs(nullptr, tb, key.as<uint32_t>(), key_o.as<uint32_t>(),
                                     val.as<int32_t>(), gperm.as<int32_t>(), (size_t)n, 0u,
                                     end_bit, s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tb, key.as<uint32_t>(), key_o.as<uint32_t>(),
                                     val.as<int32_t>(), gperm.as<int32_t>(), (size_t)n, 0u,
                                     end_bit, s));
    std::vector<int32_t> hc(nb);
    MM_HIP(hipMemcpyAsync(hc.data(), cnt.ptr, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    key.release();
    key_o.release();
    val.release();

    std::vector<int64_t> goff(nb + 1, 0);
    for (int32_t b = 0; b < nb; ++b) goff[b + 1] = goff[b] + hc[b];
    const int64_t nv = goff[nb];
    // waves: per group of 64 bins, ceil(largest bin / GB_CHUNK) chunks; the
    // width of a wave is its largest lane count
    const int32_t ng = (nb + 63) / 64;
    std::vector<int32_t> first(ng + 1, 0), wgroup;
    std::vector<int64_t> base(1, 0);
    for (int32_t g = 0; g < ng; ++g) {
        first[g] = (int32_t)wgroup.size();
        int64_t mx = 0;
        for (int32_t b = g * 64; b < std::min(nb, g * 64 + 64); ++b) mx = std::max<int64_t>(mx, hc[b]);
        for (int64_t k = 0; k * GB_CHUNK < mx; ++k) {
            int64_t wd = 0;
            for (int32_t b = g * 64; b < std::min(nb, g * 64 + 64); ++b)
                wd = std::max<int64_t>(wd, std::min<int64_t>(GB_CHUNK, hc[b] - k * GB_CHUNK));
            wgroup.push_back(g);
            base.push_back(base.back() + 64 * wd);
        }
    }
    first[ng] = (int32_t)wgroup.size();
    const int32_t n_wave = (int32_t)wgroup.size();
    nz->pf_nb = nb;
    nz->pf_n_gwave = n_wave;
    DBuf goff_d, gperm_d, gw_d, wgroup_d;
    goff_d.alloc(sizeof(int64_t) * (nb + 1));
    gw_d.alloc(sizeof(double) * (nv > 0 ? nv : 1));
    wgroup_d.alloc(sizeof(int32_t) * (n_wave > 0 ? n_wave : 1));
    nz->pf_gbase.alloc(sizeof(int64_t) * base.size());
    nz->pf_gfirst.alloc(sizeof(int32_t) * (ng + 1));
    nz->pf_gsp.alloc(sizeof(int32_t) * (base.back() > 0 ? base.back() : 1));
    nz->pf_gsw.alloc(sizeof(double) * (base.back() > 0 ? base.back() : 1));
    nz->pf_gwinv.alloc(sizeof(double) * nb);
    MM_HIP(hipMemcpyAsync(goff_d.ptr, goff.data(), sizeof(int64_t) * (nb + 1),
                          hipMemcpyHostToDevice, s));
    MM_HIP(hipMemcpyAsync(nz->pf_gbase.ptr, base.data(), sizeof(int64_t) * base.size(),
                          hipMemcpyHostToDevice, s));
    MM_HIP(hipMemcpyAsync(nz->pf_gfirst.ptr, first.data(), sizeof(int32_t) * (ng + 1),
                          hipMemcpyHostToDevice, s));
    if (n_wave > 0)
        MM_HIP(hipMemcpyAsync(wgroup_d.ptr, wgroup.data(), sizeof(int32_t) * n_wave,
                              hipMemcpyHostToDevice, s));
    if (nv > 0)
        k_gb_weights<<<grid_for(nv), BS, 0, s>>>(gperm.as<int32_t>(), nv,
                                                 nz->pf_sub.as<int64_t>(), nz->pf_n_sub,
                                                 nz->pf_omega.as<double>(),
                                                 nz->pf_mask.as<uint32_t>(), gw_d.as<double>());
    k_gb_winv<<<(unsigned)(((int64_t)nb * 64 + BS - 1) / BS), BS, 0, s>>>(
        goff_d.as<int64_t>(), nb, gw_d.as<double>(), nz->pf_gwinv.as<double>());
    if (n_wave > 0)
        k_gb_fill<<<(unsigned)std::min<int64_t>(((int64_t)n_wave * 64 + BS - 1) / BS, 16384), BS,
                    0, s>>>(nz->pf_gbase.as<int64_t>(), n_wave, wgroup_d.as<int32_t>(),
                            nz->pf_gfirst.as<int32_t>(), goff_d.as<int64_t>(), nb,
                            gperm.as<int32_t>(), gw_d.as<double>(), nz->pf_gsp.as<int32_t>(),
                            nz->pf_gsw.as<double>());
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(s));
}

}  // namespace

int polyfilter_max_order() { return PF_MAX_ORDER; }

void polyfilter_prepare(mm_ctx *ctx, const mm_pointing *p, mm_noise *nz,
                        const int32_t *ground_bin, int32_t n_ground_bins) {
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
    if (ground_bin) ground_prepare(ctx, nz, ground_bin, n_ground_bins);
}

size_t polyfilter_scratch_bytes(const mm_noise *nz, int nrhs) {
    if (nz->pf_nb == 0) return 0;
    const size_t te = nz->prec == MM_F32 ? sizeof(float) : sizeof(double);
    const size_t n_part = (size_t)(nz->pf_n_gwave > 0 ? nz->pf_n_gwave : 1) * nrhs * 64;
    const size_t n_ghat = (size_t)nz->pf_nb * nrhs;
    return (te * (size_t)nz->n_samp * nrhs + 255) / 256 * 256 + te * (n_part + n_ghat);
}

void polyfilter_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z,
                          char *scratch) {
    Scope sc(ctx->prof, ctx->stream, "Ninv_poly");
    const int NP = nz->pf_order + 1;
    hipStream_t s = ctx->stream;
    dim3 grid((unsigned)((nz->pf_n_sub * 64 + BS - 1) / BS), nrhs);
    const bool f32 = nz->prec == MM_F32;
    const size_t te = f32 ? sizeof(float) : sizeof(double);
    auto run = [&](auto TT, const void *in, const void *gh, bool weighted, void *out) {
        using T = decltype(TT);
        dispatch_np(NP, [&](auto NN) {
            constexpr int N = decltype(NN)::value;
            // the register cache that holds the longest subscan (one kernel
            // per size: a kernel's registers are those of its largest path)
            auto go = [&](auto VV) {
                k_pf_apply<T, N, decltype(VV)::value><<<grid, BS, 0, s>>>(
                    nz->pf_sub.as<int64_t>(), nz->pf_omega.as<double>(), nz->pf_n_sub,
                    nz->pf_mask.as<uint32_t>(), nz->pf_ginv.as<double>(), nrhs,
                    static_cast<const T *>(in), gh ? nz->pf_gbin.as<int32_t>() : nullptr,
                    static_cast<const T *>(gh), weighted, static_cast<T *>(out));
            };
            if (nz->pf_max_len <= 256) go(std::integral_constant<int, 4>());
            else if (nz->pf_max_len <= 512) go(std::integral_constant<int, 8>());
            else go(std::integral_constant<int, 0>());
        });
    };
    auto ground = [&](auto TT, const void *y1, void *part, void *ghat) {
        using T = decltype(TT);
        if (nz->pf_n_gwave > 0)
            k_gb_part<T><<<dim3((unsigned)(((int64_t)nz->pf_n_gwave * 64 + BS - 1) / BS), nrhs),
                           BS, 0, s>>>(nz->pf_gbase.as<int64_t>(), nz->pf_n_gwave,
                                       nz->pf_gsp.as<int32_t>(), nz->pf_gsw.as<double>(), nrhs,
                                       static_cast<const T *>(y1), static_cast<T *>(part));
        const int64_t ne = (int64_t)nz->pf_nb * nrhs;
        k_gb_final<T><<<(unsigned)((ne + BS - 1) / BS), BS, 0, s>>>(
            nz->pf_gfirst.as<int32_t>(), nz->pf_nb, nz->pf_gwinv.as<double>(), nrhs,
            static_cast<const T *>(part), static_cast<T *>(ghat));
    };
    if (nz->pf_nb == 0) {
        if (f32) run(0.f, y, nullptr, true, z);
        else run(0.0, y, nullptr, true, z);
        MM_HIP(hipGetLastError());
        return;
    }
    // scratch: the filtered TOD y1, then the ground chunk sums and amplitudes
    const size_t n_part = (size_t)(nz->pf_n_gwave > 0 ? nz->pf_n_gwave : 1) * nrhs * 64;
    const size_t n_ghat = (size_t)nz->pf_nb * nrhs;
    const size_t y1_bytes = (te * (size_t)nz->n_samp * nrhs + 255) / 256 * 256;
    if (!scratch) {
        ws_alloc(ctx, ctx->tod_c, polyfilter_scratch_bytes(nz, nrhs));
        scratch = static_cast<char *>(ctx->tod_c.ptr);
    }
    void *y1 = scratch;
    char *part = scratch + y1_bytes;
    char *ghat = part + te * n_part;
    if (f32) {
        run(0.f, y, nullptr, false, y1);
        ground(0.f, y1, part, ghat);
        run(0.f, y1, ghat, true, z);
    } else {
        run(0.0, y, nullptr, false, y1);
        ground(0.0, y1, part, ghat);
        run(0.0, y1, ghat, true, z);
    }
    MM_HIP(hipGetLastError());
}

}  // namespace mm
