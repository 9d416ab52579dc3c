// Time-domain operators: P (map -> TOD gather), P^T (pixel-sorted segmented
// reduction, no float atomics), the banded-Toeplitz N^-1 applied directly,
// and the flag mask applied to the data.  The FFT form of N^-1 lives in
// noise_fft.hip.
//
// Layouts: map x[(3 j + a) R + r] (FP64); TOD y[t R + r] (T = float or double).
// A wavefront's 64 lanes are split into G = 64 / R sample groups of R columns,
// so one wave step touches G consecutive samples x R columns: contiguous TOD
// rows.  Each column is computed with the same arithmetic and order whatever
// the other columns hold.
#include <functional>
#include <type_traits>

#include "mm_internal.h"
#include "pol_weights.h"
#include "xcd.h"

namespace mm {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };


namespace {

constexpr int BS = 256;

template <typename T>
__global__ void __launch_bounds__(BS) k_zero(int64_t n, T *__restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n; e += (int64_t)gridDim.x * BS)
        y[e] = (T)0;
}

template <typename T, int R>
__device__ __forceinline__ T p_gather(int32_t j, typename Vec2<T>::type ww,
                                      const double *__restrict__ x, int r) {
    // branch-free: an unobserved sample (j < 0) reads pixel 0 and yields 0,
    // so the gathers of several samples are in flight together (the map is
    // never empty here)
    const double *xp = x + (int64_t)3 * (j < 0 ? 0 : j) * R + r;
    const T v = (T)xp[0] + ww.x * (T)xp[R] + ww.y * (T)xp[2 * R];
    return j < 0 ? (T)0 : v;
}

// y = P x.  Each wave step covers G = 64/R consecutive samples x R columns;
// four steps are issued together so each lane has four pixel-index loads and
// twelve map gathers in flight.
template <typename T, int R>
__global__ void __launch_bounds__(BS) k_apply_P(const int32_t *__restrict__ jpix,
                                                const typename Vec2<T>::type *__restrict__ w,
                                                int64_t n, const double *__restrict__ x,
                                                T *__restrict__ y) {
    constexpr int G = 64 / R;
    const int lane = threadIdx.x & 63;
    const int sub = lane / R, r = lane % R;
    const int64_t wave = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * BS) >> 6;
    const int64_t step = nwave * G;
    int64_t t = wave * G + sub;
    for (; t + 3 * step < n; t += 4 * step) {
        int32_t j[4];
        typename Vec2<T>::type ww[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            j[q] = jpix[t + q * step];
            ww[q] = w[t + q * step];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) y[(t + q * step) * R + r] = p_gather<T, R>(j[q], ww[q], x, r);
    }
    for (; t < n; t += step) y[t * R + r] = p_gather<T, R>(jpix[t], w[t], x, r);
}

// Single column: the map is first packed as 32-byte records (I, Q, U, 0) so
// each sample's gather is two aligned 16-byte loads instead of three 8-byte
// ones.
// 32-byte records (I, Q, U, 0) at each of the n_copies slots of every pixel
// (slot = NULL: one copy at the compact id).
__global__ void __launch_bounds__(BS) k_pack_map(const double *__restrict__ x, int32_t n_obs,
                                                 int n_copies, const int32_t *__restrict__ slot,
                                                 double2 *__restrict__ x4) {
    for (int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x; j < n_obs;
         j += (int64_t)gridDim.x * BS) {
        const double2 iq = make_double2(x[3 * j], x[3 * j + 1]);
        const double2 u0 = make_double2(x[3 * j + 2], 0.0);
        for (int g = 0; g < n_copies; ++g) {
            const int64_t s = slot ? slot[(int64_t)g * n_obs + j] : j;
            x4[2 * s] = iq;
            x4[2 * s + 1] = u0;
        }
    }
}

template <typename T>
__device__ __forceinline__ T p_gather4(int32_t j, typename Vec2<T>::type ww,
                                       const double2 *__restrict__ x4) {
    const int64_t jj = j < 0 ? 0 : j;  // branch-free, as p_gather
    const double2 iq = x4[2 * jj];
    const double u = x4[2 * jj + 1].x;
    const T v = (T)iq.x + ww.x * (T)iq.y + ww.y * (T)u;
    return j < 0 ? (T)0 : v;
}

// A once-read stream element loaded with the non-temporal cache policy: a
// double, or a float2 moved as one 64-bit word.
__device__ __forceinline__ double nt_load_w(const double *p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ float2 nt_load_w(const float2 *p) {
    return __builtin_bit_cast(
        float2, __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p)));
}
__device__ __forceinline__ double2 nt_load_w(const double2 *p) { return *p; }

template <typename T>
__global__ void __launch_bounds__(BS) k_apply_P1(const int32_t *__restrict__ jpix,
                                                 const typename Vec2<T>::type *__restrict__ w,
                                                 int64_t n, const double2 *__restrict__ x4,
                                                 T *__restrict__ y) {
    const int64_t step = (int64_t)gridDim.x * BS;
    int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
    for (; t + 7 * step < n; t += 8 * step) {
        int32_t j[8];
        typename Vec2<T>::type ww[8];
        // slots and weights are read once, and y written once: non-temporal,
        // so that they do not push the gathered map lines out of the L2
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            j[q] = __builtin_nontemporal_load(jpix + t + q * step);
            ww[q] = nt_load_w(w + t + q * step);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            __builtin_nontemporal_store(p_gather4<T>(j[q], ww[q], x4), y + t + q * step);
    }
    for (; t < n; t += step) y[t] = p_gather4<T>(jpix[t], w[t], x4);
}

// Single column, FP64: the weights are formed from the stored angles, so a
// sample costs its map slot and angle (12 bytes) instead of index and two
// weights (20 bytes).  The map is split into I (8 bytes) and (Q, U) (16
// bytes) per slot; with a grid the slots follow Morton order, so the pixels
// of 64 consecutive samples fall in few cache lines whatever the scan
// direction.  Same arithmetic and order as k_apply_P (bitwise the same y).
// Split map for P: I in xi, (Q, U) in xqu, at each of the n_copies slots of
// every pixel (slot = NULL: one copy at the compact id).
__global__ void __launch_bounds__(BS) k_pack_map_split(const double *__restrict__ x,
                                                       int32_t n_obs, int n_copies,
                                                       const int32_t *__restrict__ slot,
                                                       double *__restrict__ xi,
                                                       double2 *__restrict__ xqu) {
    for (int64_t c = (int64_t)blockIdx.x * BS + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * BS) {
        const double vi = x[3 * c];
        const double2 vqu = make_double2(x[3 * c + 1], x[3 * c + 2]);
        for (int g = 0; g < n_copies; ++g) {
            const int64_t s = slot ? slot[(int64_t)g * n_obs + c] : c;
            xi[s] = vi;
            xqu[s] = vqu;
        }
    }
}

__device__ __forceinline__ double p_gather_psi(int32_t j, double psi,
                                               const double *__restrict__ xi,
                                               const double2 *__restrict__ xqu) {
    const int32_t jj = j < 0 ? 0 : j;  // branch-free, as p_gather
    const double i0 = xi[jj];
    const double2 qu = xqu[jj];
    double c, s;
    pol_weights(psi, c, s);
    const double v = i0 + c * qu.x + s * qu.y;
    return j < 0 ? 0.0 : v;
}

__global__ void __launch_bounds__(BS) k_apply_P1_psi(const int32_t *__restrict__ jpix,
                                                     const double *__restrict__ psi, int64_t n,
                                                     const double *__restrict__ xi,
                                                     const double2 *__restrict__ xqu,
                                                     double *__restrict__ y) {
    const int64_t step = (int64_t)gridDim.x * BS;
    int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
    // eight samples in flight per thread (measured: 0.70 ms against 0.73 with
    // four at 1.34e8 samples; sixteen gave no more): their slots and angles,
    // then their eight map gathers (from slot 0 where the sample is
    // unobserved, so that no gather waits behind a branch), then the weights
    for (; t + 7 * step < n; t += 8 * step) {
        int32_t j[8];
        double a[8], i8[8];
        double2 qu8[8];
        // slots and angles are read once, and y written once: non-temporal,
        // so that they do not push the gathered map lines out of the L2
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            j[q] = __builtin_nontemporal_load(jpix + t + q * step);
            a[q] = __builtin_nontemporal_load(psi + t + q * step);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int32_t jj = j[q] < 0 ? 0 : j[q];
            i8[q] = xi[jj];
            qu8[q] = xqu[jj];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double c, s;
            pol_weights(a[q], c, s);
            const double v = i8[q] + c * qu8[q].x + s * qu8[q].y;
            __builtin_nontemporal_store(j[q] < 0 ? 0.0 : v, y + t + q * step);
        }
    }
    for (; t < n; t += step) y[t] = p_gather_psi(jpix[t], psi[t], xi, xqu);
}

// Pixels are visited in the order `order` (NULL = ascending), e.g. square
// tiles of the map, and each XCD takes a contiguous range of that order: the
// pixels one XCD reduces together are neighbours, hit by the same stretches of
// the scan, so their gathers of z share cache lines in that XCD's L2.
template <typename T, int R>
__global__ void __launch_bounds__(BS) k_apply_PT(const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ perm,
                                                 const typename Vec2<T>::type *__restrict__ ws,
                                                 int32_t n_obs, const int32_t *__restrict__ order,
                                                 const T *__restrict__ z,
                                                 double *__restrict__ x) {
    constexpr int G = 64 / R;
    const int lane = threadIdx.x & 63;
    const int sub = lane / R, r = lane % R;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t s = blk * (BS / 64) + (threadIdx.x >> 6);
    if (s >= n_obs) return;
    const int64_t j = order ? order[s] : s;
    const int32_t a = off[j], b = off[j + 1];
    T s0 = 0, s1 = 0, s2 = 0;
    int32_t i = a + sub;
    // four entries in flight per lane, accumulated in segment order
    for (; i + 3 * G < b; i += 4 * G) {
        int32_t tt[4];
        T zz[4];
        typename Vec2<T>::type ww[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) tt[q] = perm[i + q * G];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            zz[q] = z[(int64_t)tt[q] * R + r];
            ww[q] = ws[i + q * G];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            s0 += zz[q];
            s1 += ww[q].x * zz[q];
            s2 += ww[q].y * zz[q];
        }
    }
    for (; i < b; i += G) {
        const int32_t tq = perm[i];
        const T zq = z[(int64_t)tq * R + r];
        const auto wq = ws[i];
        s0 += zq;
        s1 += wq.x * zq;
        s2 += wq.y * zq;
    }
#pragma unroll
    for (int m = 32; m >= R; m >>= 1) {
        s0 += __shfl_xor(s0, m);
        s1 += __shfl_xor(s1, m);
        s2 += __shfl_xor(s2, m);
    }
    if (sub == 0) {
        double *xp = x + (int64_t)3 * j * R + r;
        xp[0] = (double)s0;
        xp[R] = (double)s1;
        xp[2 * R] = (double)s2;
    }
}

// Sliced single-column P^T.  Wave w = s G + g (remapped so that each XCD takes
// a contiguous range of w) owns 64 pixels (one per lane) and time segment s;
// every lane walks its pixel's entries of that segment in time order and
// accumulates in registers.  Lanes hold neighbouring pixels, and all waves
// are resident together, so the whole grid advances through the TOD at a
// similar pace and the lines of z it gathers are shared in L2 and the
// Infinity Cache instead of re-read from HBM.  Partial maps per segment go to
// part[s][3 c + a] (or straight to x when S = 1).
// Weight record of an entry: FP64 stores the angle and forms the weights
// here; FP32 stores the two weights.
template <typename T> struct SlRec;
template <> struct SlRec<double> {
    using type = double;
    __device__ static void weights(double psi, double &c, double &s) { pol_weights(psi, c, s); }
};
template <> struct SlRec<float> {
    using type = float2;
    __device__ static void weights(float2 w, float &c, float &s) {
        c = w.x;
        s = w.y;
    }
};

template <typename T>
__global__ void __launch_bounds__(BS) k_apply_PT_sl(const int64_t *__restrict__ base,
                                                    const int32_t *__restrict__ sl_perm,
                                                    const typename SlRec<T>::type *__restrict__ sl_w,
                                                    const int32_t *__restrict__ sl_pix, int32_t G,
                                                    int32_t S, int32_t n_obs,
                                                    const T *__restrict__ z,
                                                    double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t w = blk * (BS / 64) + (threadIdx.x >> 6);
    if (w >= (int64_t)G * S) return;
    const int32_t sg = (int32_t)(w / G), g = (int32_t)(w % G);
    const int64_t b0 = base[w];
    const int64_t W = (base[w + 1] - b0) >> 6;
    const int32_t *pp = sl_perm + b0 + lane;
    const auto *wp = sl_w + b0 + lane;
    T s0 = 0, s1 = 0, s2 = 0;
    int64_t k = 0;
    // eight entries in flight per lane, accumulated in entry order
    for (; k + 7 < W; k += 8) {
        int32_t tt[8];
        typename SlRec<T>::type ww[8];
        T zz[8];
        // the sample indices and weights are read once: non-temporal, so
        // that they do not push the gathered z lines out of the L2
#pragma unroll
        for (int q = 0; q < 8; ++q) tt[q] = __builtin_nontemporal_load(pp + 64 * (k + q));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            ww[q] = nt_load_w(wp + 64 * (k + q));
            // a padding entry (-1) reads sample 0 and adds 0: no branch
            // between the eight gathers
            const T zq = z[tt[q] < 0 ? 0 : tt[q]];
            zz[q] = tt[q] >= 0 ? zq : (T)0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            T c, sn;
            SlRec<T>::weights(ww[q], c, sn);
            s0 += zz[q];
            s1 += c * zz[q];
            s2 += sn * zz[q];
        }
    }
    for (; k < W; ++k) {
        const int32_t tq = pp[64 * k];
        T c, sn;
        SlRec<T>::weights(wp[64 * k], c, sn);
        const T zq = tq >= 0 ? z[tq] : (T)0;
        s0 += zq;
        s1 += c * zq;
        s2 += sn * zq;
    }
    const int32_t c = sl_pix[(int64_t)g * 64 + lane];
    if (c < 0) return;
    double *o = out + ((int64_t)sg * n_obs + c) * 3;
    o[0] = (double)s0;
    o[1] = (double)s1;
    o[2] = (double)s2;
}

// x[e] = part[0][e] + part[1][e] + ... in segment order; the partials' loads
// are issued eight at a time (a runtime-length loop would wait for each).
__global__ void __launch_bounds__(BS) k_pt_sum_parts(const double *__restrict__ part, int32_t S,
                                                     int64_t n3, double *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n3;
         e += (int64_t)gridDim.x * BS) {
        double acc = part[e];
        int32_t sg = 1;
        for (; sg + 7 < S; sg += 8) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[(sg + q) * n3 + e];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += v[q];
        }
        for (; sg < S; ++sg) acc += part[sg * n3 + e];
        x[e] = acc;
    }
}

// Pointings of the pair-sum (I, NC = 1: weight 1) and pair-difference (QU,
// NC = 2: weights cos 2psi, sin 2psi) streams (Eqs. d+ and d-).  Same
// structure as k_apply_P / k_apply_PT; map x[(NC j + a) R + r].
template <typename T, int R, int NC>
__device__ __forceinline__ T p_gather_nc(int32_t j, typename Vec2<T>::type ww,
                                         const double *__restrict__ x, int r) {
    if (j < 0) return (T)0;
    const double *xp = x + (int64_t)NC * j * R + r;
    if constexpr (NC == 1) return (T)xp[0];
    else return ww.x * (T)xp[0] + ww.y * (T)xp[R];
}

template <typename T, int R, int NC>
__global__ void __launch_bounds__(BS) k_apply_P_nc(const int32_t *__restrict__ jpix,
                                                   const typename Vec2<T>::type *__restrict__ w,
                                                   int64_t n, const double *__restrict__ x,
                                                   T *__restrict__ y) {
    constexpr int G = 64 / R;
    const int lane = threadIdx.x & 63;
    const int sub = lane / R, r = lane % R;
    const int64_t wave = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * BS) >> 6;
    const int64_t step = nwave * G;
    for (int64_t t = wave * G + sub; t < n; t += step) {
        typename Vec2<T>::type ww{};
        if constexpr (NC == 2) ww = w[t];
        y[t * R + r] = p_gather_nc<T, R, NC>(jpix[t], ww, x, r);
    }
}

template <typename T, int R, int NC>
__global__ void __launch_bounds__(BS) k_apply_PT_nc(const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ perm,
                                                    const typename Vec2<T>::type *__restrict__ ws,
                                                    int32_t n_obs,
                                                    const int32_t *__restrict__ order,
                                                    const T *__restrict__ z,
                                                    double *__restrict__ x) {
    constexpr int G = 64 / R;
    const int lane = threadIdx.x & 63;
    const int sub = lane / R, r = lane % R;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t s = blk * (BS / 64) + (threadIdx.x >> 6);
    if (s >= n_obs) return;
    const int64_t j = order ? order[s] : s;
    const int32_t a = off[j], b = off[j + 1];
    T s0 = 0, s1 = 0;
    for (int32_t i = a + sub; i < b; i += G) {
        const T zq = z[(int64_t)perm[i] * R + r];
        if constexpr (NC == 1) {
            s0 += zq;
        } else {
            const auto wq = ws[i];
            s0 += wq.x * zq;
            s1 += wq.y * zq;
        }
    }
#pragma unroll
    for (int m = 32; m >= R; m >>= 1) {
        s0 += __shfl_xor(s0, m);
        if constexpr (NC == 2) s1 += __shfl_xor(s1, m);
    }
    if (sub == 0) {
        double *xp = x + (int64_t)NC * j * R + r;
        xp[0] = (double)s0;
        if constexpr (NC == 2) xp[R] = (double)s1;
    }
}

// plus = (a + b) / 2, minus = (a - b) / 2 (either output may be null; an
// output may be one of the inputs, as each element is read before it is
// written).
template <typename T>
__global__ void __launch_bounds__(BS) k_sum_diff(int64_t n, const T *a, const T *b, T *plus,
                                                 T *minus) {
    for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * BS) {
        const T u = a[t], v = b[t];
        if (plus) plus[t] = (u + v) * (T)0.5;
        if (minus) minus[t] = (u - v) * (T)0.5;
    }
}

// Direct band, register-tiled.  A block owns TL = (BS / R) * BT_OPT
// consecutive outputs of one interval for all R columns; thread (g, r) =
// (threadIdx / R, threadIdx mod R) keeps outputs g*BT_OPT .. g*BT_OPT + 7 of
// column r in registers.  The filter is taken as the full symmetric one,
// f[d] = c_|d - lambda|, d = 0 .. 2 lambda, and walked in chunks of at most
// CL taps; for each chunk the taps and the input window [t0 - lambda + d0,
// t0 + TL - lambda + d0 + CL - 1) (zero outside the interval, R values per
// row, so a wave's reads are consecutive) are staged in LDS.  Per block of
// BT_OPT taps a thread loads 15 inputs and 8 taps and does 64 FMAs from
// registers.  Every output sums its taps in ascending offset, chunk after
// chunk, so its value does not depend on R, TL or CL; zero-padded terms add
// exactly +0.
constexpr int BT_OPT = 8;
constexpr int BT_LDS = 65536;  // bytes of LDS per block
// One column on a short stream (nz->band_small): blocks of 64 threads, tiles
// of 512 outputs, so that the few tiles of such a stream still spread over
// the CUs (config 1's 131,072 samples: 256 blocks instead of 64).
constexpr int BAND_SMALL_NT = 64;

template <typename T, int R, int NT = BS>
__global__ void __launch_bounds__(NT) k_band_tiled(const int64_t *__restrict__ pref, int n_int,
                                                   const int64_t *__restrict__ istart,
                                                   const int32_t *__restrict__ fid,
                                                   const T *__restrict__ band, int lam, int CL,
                                                   const T *__restrict__ y, T *__restrict__ z) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TL = (NT / R) * BT_OPT;
    const int nf = 2 * lam + 1;
    const int nf_pad = (nf + BT_OPT - 1) / BT_OPT * BT_OPT;
    // CL is a multiple of BT_OPT; rounding it here lets the compiler see
    // that the window is 16-byte aligned and read it with 128-bit LDS loads
    const int CLa = CL / BT_OPT * BT_OPT;
    T *sf = reinterpret_cast<T *>(smem_raw);  // CL taps
    T *sy = sf + CLa;                          // (TL + CL - 1) rows of R
    // tile -> interval: pref[i] counts the tiles of intervals before i
    const int64_t bt = blockIdx.x;
    int lo = 0, hi = n_int;  // pref[lo] <= bt < pref[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= bt) lo = mid; else hi = mid;
    }
    const int64_t iv = lo;
    const int64_t a = istart[iv], b = istart[iv + 1];
    const int64_t t0 = a + (bt - pref[iv]) * TL;
    const T *c = band + (int64_t)fid[iv] * (lam + 1);
    const int r = threadIdx.x % R;
    const int m0 = (threadIdx.x / R) * BT_OPT;
    T acc[BT_OPT];
#pragma unroll
    for (int m = 0; m < BT_OPT; ++m) acc[m] = 0;
    for (int d0 = 0; d0 < nf_pad; d0 += CLa) {
        const int cl = nf_pad - d0 < CLa ? nf_pad - d0 : CLa;
        __syncthreads();  // the previous chunk's reads are done
        // The staging loads are issued eight per thread at a time: each
        // address is clamped to a valid element (tap 0, or the interval's
        // first sample) and the value zeroed where it falls outside, so no
        // load waits behind a branch.  The staged values are the same.
        int k = threadIdx.x;
        for (; k + 7 * NT < cl; k += 8 * NT) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int ku = k + u * NT;
                const int d = d0 + ku - lam;
                const bool in = d0 + ku < nf;
                v[u] = c[in ? (d < 0 ? -d : d) : 0];
                v[u] = in ? v[u] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) sf[k + u * NT] = v[u];
        }
        for (; k < cl; k += NT) {
            const int d = d0 + k - lam;
            sf[k] = d0 + k < nf ? c[d < 0 ? -d : d] : (T)0;
        }
        const int rows = TL + cl - 1;
        const int64_t w0 = t0 - lam + d0;
        int e = threadIdx.x;
        for (; e + 7 * NT < rows * R; e += 8 * NT) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int eu = e + u * NT;
                const int64_t t = w0 + eu / R;
                const bool in = t >= a && t < b;
                v[u] = y[(in ? t : a) * R + eu % R];
                v[u] = in ? v[u] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) sy[e + u * NT] = v[u];
        }
        for (; e < rows * R; e += NT) {
            const int64_t t = w0 + e / R;
            sy[e] = (t >= a && t < b) ? y[t * R + e % R] : (T)0;
        }
        __syncthreads();
        for (int db = 0; db < cl; db += BT_OPT) {
            T w[2 * BT_OPT - 1], cf[BT_OPT];
#pragma unroll
            for (int q = 0; q < 2 * BT_OPT - 1; ++q) w[q] = sy[(m0 + db + q) * R + r];
#pragma unroll
            for (int q = 0; q < BT_OPT; ++q) cf[q] = sf[db + q];
#pragma unroll
            for (int q = 0; q < BT_OPT; ++q)
#pragma unroll
                for (int m = 0; m < BT_OPT; ++m) acc[m] += cf[q] * w[m + q];
        }
    }
    const int64_t t1 = t0 + TL < b ? t0 + TL : b;
#pragma unroll
    for (int m = 0; m < BT_OPT; ++m) {
        const int64_t t = t0 + m0 + m;
        if (t < t1) z[t * R + r] = acc[m];
    }
}

// y[t R + r] = mask_t * tod[r * n + t]; flags non-finite data on kept samples.
template <typename T, int R>
__global__ void __launch_bounds__(BS) k_mask(const int32_t *__restrict__ jpix, int64_t n,
                                             const T *__restrict__ tod, T *__restrict__ y,
                                             int *__restrict__ flag) {
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n * R;
         e += (int64_t)gridDim.x * BS) {
        const int64_t t = e / R;
        const int r = (int)(e % R);
        T v = tod[(int64_t)r * n + t];
        if (jpix[t] >= 0) {
            bad |= !isfinite(v);
        } else {
            v = (T)0;
        }
        y[e] = v;
    }
    if (bad) atomicOr(flag, 1);
}

int grid_for(int64_t n, int max_blocks = 16384) {
    int64_t g = (n + BS - 1) / BS;
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

template <typename F> void dispatch_r(int nrhs, F &&f) {
    switch (nrhs) {
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        case 8: f(std::integral_constant<int, 8>()); break;
        case 16: f(std::integral_constant<int, 16>()); break;
        case 32: f(std::integral_constant<int, 32>()); break;
        case 64: f(std::integral_constant<int, 64>()); break;
        default: throw Error(MM_E_INVALID, "nrhs must be a power of two <= 64");
    }
}

}  // namespace

void apply_P_dev(mm_ctx *ctx, const mm_pointing *p, int nrhs, const double *x, void *y,
                 char *scratch) {
    Scope sc(ctx->prof, ctx->stream, "P");
    const int64_t n = p->n_samp;
    if (p->n_obs == 0) {  // no observed pixel: y = 0 (the gathers assume a pixel 0)
        const int64_t ne = n * nrhs;
        if (ne > 0) {
            if (p->prec == MM_F32)
                k_zero<float><<<grid_for(ne), BS, 0, ctx->stream>>>(ne, static_cast<float *>(y));
            else
                k_zero<double><<<grid_for(ne), BS, 0, ctx->stream>>>(ne, static_cast<double *>(y));
            MM_HIP(hipGetLastError());
        }
        return;
    }
    if (p->nc != 3) {
        dispatch_r(nrhs, [&](auto RR) {
            constexpr int R = decltype(RR)::value;
            const int grid = grid_for(n * R, 8 * ctx->n_cu * 4);
            auto go = [&](auto TT, auto NN) {
                using T = decltype(TT);
                constexpr int NC = decltype(NN)::value;
                k_apply_P_nc<T, R, NC><<<grid, BS, 0, ctx->stream>>>(
                    p->j.as<int32_t>(),
                    NC == 2 ? static_cast<const typename Vec2<T>::type *>(p->w.ptr) : nullptr, n,
                    x, static_cast<T *>(y));
            };
            if (p->prec == MM_F32) {
                if (p->nc == 1) go(0.f, std::integral_constant<int, 1>());
                else go(0.f, std::integral_constant<int, 2>());
            } else {
                if (p->nc == 1) go(0.0, std::integral_constant<int, 1>());
                else go(0.0, std::integral_constant<int, 2>());
            }
        });
        MM_HIP(hipGetLastError());
        return;
    }
    if (nrhs == 1) {
        const bool slots = p->p_j.ptr != nullptr;
        const int copies = slots ? p->p_copies : 1;
        const size_t no = (size_t)(p->n_obs > 0 ? p->n_obs : 1) * copies;
        if (!scratch) {
            ws_alloc(ctx, ctx->xpack, apply_P_scratch_bytes(p, nrhs));
            scratch = static_cast<char *>(ctx->xpack.ptr);
        }
        double2 *xpack = reinterpret_cast<double2 *>(scratch);
        const int tuned = p->p_blocks[0];
        if (p->prec == MM_F32) {
            k_pack_map<<<grid_for(p->n_obs, 1024), BS, 0, ctx->stream>>>(
                x, p->n_obs, copies, slots ? p->p_slot.as<int32_t>() : nullptr, xpack);
            const int grid = tuned > 0 ? tuned : grid_for(n, 8 * ctx->n_cu * 4);
            k_apply_P1<float><<<grid, BS, 0, ctx->stream>>>(
                slots ? p->p_j.as<int32_t>() : p->j.as<int32_t>(), p->w.as<float2>(), n, xpack,
                static_cast<float *>(y));
        } else {
            // xpack holds I (no doubles) then (Q, U) (no double2), no = n_obs x copies
            double *xi = reinterpret_cast<double *>(scratch);
            double2 *xqu = reinterpret_cast<double2 *>(xi + 2 * ((no + 1) / 2));
            k_pack_map_split<<<grid_for(p->n_obs, 1024), BS, 0, ctx->stream>>>(
                x, p->n_obs, copies, slots ? p->p_slot.as<int32_t>() : nullptr, xi, xqu);
            const int grid = tuned > 0 ? tuned : grid_for(n, 32 * ctx->n_cu * 4);
            k_apply_P1_psi<<<grid, BS, 0, ctx->stream>>>(
                slots ? p->p_j.as<int32_t>() : p->j.as<int32_t>(), p->psi.as<double>(), n, xi, xqu,
                static_cast<double *>(y));
        }
        MM_HIP(hipGetLastError());
        return;
    }
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        const int tuned = p->p_blocks[log2i(R)];
        const int grid = tuned > 0 ? tuned : grid_for(n * R, 8 * ctx->n_cu * 4);
        if (p->prec == MM_F32)
            k_apply_P<float, R><<<grid, BS, 0, ctx->stream>>>(p->j.as<int32_t>(),
                                                              p->w.as<float2>(), n, x,
                                                              static_cast<float *>(y));
        else
            k_apply_P<double, R><<<grid, BS, 0, ctx->stream>>>(p->j.as<int32_t>(),
                                                               p->w.as<double2>(), n, x,
                                                               static_cast<double *>(y));
    });
    MM_HIP(hipGetLastError());
}

size_t apply_P_scratch_bytes(const mm_pointing *p, int nrhs) {
    if (p->nc != 3 || nrhs != 1) return 0;
    const int copies = p->p_j.ptr != nullptr ? p->p_copies : 1;
    return sizeof(double2) * 2 * (size_t)(p->n_obs > 0 ? p->n_obs : 1) * copies;
}

size_t apply_PT_scratch_bytes(const mm_pointing *p, int nrhs) {
    if (p->nc != 3 || nrhs != 1 || p->sl_G <= 0 || p->n_obs == 0) return 0;
    const int64_t parts = (int64_t)p->sl_S * p->sl_D;
    return parts > 1 ? sizeof(double) * (size_t)(3 * (int64_t)p->n_obs * parts) : 0;
}

void apply_PT_dev(mm_ctx *ctx, const mm_pointing *p, int nrhs, const void *z, double *x,
                  char *scratch) {
    Scope sc(ctx->prof, ctx->stream, "PT");
    if (p->n_obs == 0) return;
    if (p->nc != 3) {
        int64_t nb = (p->n_obs + 3) / 4;
        if (nb >= 64) nb = (nb + 7) & ~(int64_t)7;
        const int32_t *order = p->seg_order.ptr ? p->seg_order.as<int32_t>() : nullptr;
        dispatch_r(nrhs, [&](auto RR) {
            constexpr int R = decltype(RR)::value;
            auto go = [&](auto TT, auto NN) {
                using T = decltype(TT);
                constexpr int NC = decltype(NN)::value;
                k_apply_PT_nc<T, R, NC><<<(unsigned)nb, BS, 0, ctx->stream>>>(
                    p->off.as<int32_t>(), p->perm.as<int32_t>(),
                    NC == 2 ? static_cast<const typename Vec2<T>::type *>(p->ws.ptr) : nullptr,
                    p->n_obs, order, static_cast<const T *>(z), x);
            };
            if (p->prec == MM_F32) {
                if (p->nc == 1) go(0.f, std::integral_constant<int, 1>());
                else go(0.f, std::integral_constant<int, 2>());
            } else {
                if (p->nc == 1) go(0.0, std::integral_constant<int, 1>());
                else go(0.0, std::integral_constant<int, 2>());
            }
        });
        MM_HIP(hipGetLastError());
        return;
    }
    if (nrhs == 1 && p->sl_G > 0) {
        // lane pixels are virtual ids d n_obs + c (sl_D scan directions), so
        // wave (s, g) writes partial map s D + d; the partials are then
        // added in that fixed order
        const int32_t G = p->sl_G, S = p->sl_S, D = p->sl_D;
        const int64_t n3 = 3 * (int64_t)p->n_obs;
        const int32_t parts = S * D;
        double *out = x;
        if (parts > 1) {
            if (!scratch) {
                ws_alloc(ctx, ctx->pt_part, apply_PT_scratch_bytes(p, nrhs));
                scratch = static_cast<char *>(ctx->pt_part.ptr);
            }
            out = reinterpret_cast<double *>(scratch);
        }
        const int32_t nv = D * p->n_obs;
        int64_t nb = ((int64_t)G * S + 3) / 4;
        if (nb >= 64) nb = (nb + 7) & ~(int64_t)7;
        if (p->prec == MM_F32)
            k_apply_PT_sl<float><<<(unsigned)nb, BS, 0, ctx->stream>>>(
                p->sl_base.as<int64_t>(), p->sl_perm.as<int32_t>(), p->sl_w.as<float2>(),
                p->sl_pix.as<int32_t>(), G, S, nv, static_cast<const float *>(z), out);
        else
            k_apply_PT_sl<double><<<(unsigned)nb, BS, 0, ctx->stream>>>(
                p->sl_base.as<int64_t>(), p->sl_perm.as<int32_t>(), p->sl_w.as<double>(),
                p->sl_pix.as<int32_t>(), G, S, nv, static_cast<const double *>(z), out);
        if (parts > 1)
            k_pt_sum_parts<<<grid_for(n3, 2048), BS, 0, ctx->stream>>>(out, parts, n3, x);
        MM_HIP(hipGetLastError());
        return;
    }
    int64_t nb = (p->n_obs + 3) / 4;
    if (nb >= 64) nb = (nb + 7) & ~(int64_t)7;
    const int po = p->pt_order[log2i(nrhs)];
    const int32_t *order = (p->seg_order.ptr && po != 0) ? p->seg_order.as<int32_t>() : nullptr;
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        if (p->prec == MM_F32)
            k_apply_PT<float, R><<<(unsigned)nb, BS, 0, ctx->stream>>>(
                p->off.as<int32_t>(), p->perm.as<int32_t>(), p->ws.as<float2>(), p->n_obs, order,
                static_cast<const float *>(z), x);
        else
            k_apply_PT<double, R><<<(unsigned)nb, BS, 0, ctx->stream>>>(
                p->off.as<int32_t>(), p->perm.as<int32_t>(), p->ws.as<double2>(), p->n_obs,
                order, static_cast<const double *>(z), x);
    });
    MM_HIP(hipGetLastError());
}

void noise_fft_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z);

// Tile length of the direct band for R columns.
int band_tile_len(int nrhs, bool small) {
    return nrhs == 1 && small ? BAND_SMALL_NT * BT_OPT : (BS / nrhs) * BT_OPT;
}

// Taps per LDS chunk of the direct band: taps + window rows of R values fit
// in BT_LDS bytes; a multiple of BT_OPT, at most the padded filter length.
static int band_chunk(int lam, int R, mm_precision prec, bool small) {
    const size_t te = prec == MM_F32 ? sizeof(float) : sizeof(double);
    const int tl = band_tile_len(R, small);
    const int nf_pad = (2 * lam + 1 + BT_OPT - 1) / BT_OPT * BT_OPT;
    int cl = (int)(((int64_t)(BT_LDS / te) - (int64_t)(tl - 1) * R) / (R + 1));
    cl = cl / BT_OPT * BT_OPT;
    return cl < nf_pad ? cl : nf_pad;
}

size_t noise_scratch_bytes(const mm_noise *nz, int nrhs) {
    return nz->method == MM_NOISE_POLY ? polyfilter_scratch_bytes(nz, nrhs) : 0;
}

void noise_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z,
                     char *scratch) {
    if (nz->method == MM_NOISE_FFT) {
        noise_fft_apply_dev(ctx, nz, nrhs, y, z);
        return;
    }
    if (nz->method == MM_NOISE_POLY) {
        polyfilter_apply_dev(ctx, nz, nrhs, y, z, scratch);
        return;
    }
    Scope sc(ctx->prof, ctx->stream, "Ninv_band");
    const int lam = nz->half_bw;
    const int tl = band_tile_len(nrhs, nz->band_small);
    // tile counts for every column count are built with the noise handle, so
    // an apply never modifies it (handles may be shared across contexts)
    const int li = log2i(nrhs);
    const int64_t *pref = nz->tile_pref.as<int64_t>() + (int64_t)li * (nz->n_int + 1);
    const unsigned n_tiles = (unsigned)nz->h_tile_pref[(size_t)li * (nz->n_int + 1) + nz->n_int];
    const int cl =
        nz->band_cl[li] > 0 ? nz->band_cl[li] : band_chunk(lam, nrhs, nz->prec, nz->band_small);
    const size_t te = nz->prec == MM_F32 ? sizeof(float) : sizeof(double);
    const size_t sm = te * ((size_t)cl + (size_t)(tl + cl - 1) * nrhs);
    if (nrhs == 1 && nz->band_small) {  // short single streams: 64-thread blocks
        if (nz->prec == MM_F32)
            k_band_tiled<float, 1, BAND_SMALL_NT><<<n_tiles, BAND_SMALL_NT, sm, ctx->stream>>>(
                pref, nz->n_int, nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
                nz->band.as<float>(), lam, cl, static_cast<const float *>(y),
                static_cast<float *>(z));
        else
            k_band_tiled<double, 1, BAND_SMALL_NT><<<n_tiles, BAND_SMALL_NT, sm, ctx->stream>>>(
                pref, nz->n_int, nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
                nz->band.as<double>(), lam, cl, static_cast<const double *>(y),
                static_cast<double *>(z));
        MM_HIP(hipGetLastError());
        return;
    }
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        if (nz->prec == MM_F32)
            k_band_tiled<float, R><<<n_tiles, BS, sm, ctx->stream>>>(
                pref, nz->n_int, nz->istart.as<int64_t>(), nz->fid.as<int32_t>(), nz->band.as<float>(), lam,
                cl, static_cast<const float *>(y), static_cast<float *>(z));
        else
            k_band_tiled<double, R><<<n_tiles, BS, sm, ctx->stream>>>(
                pref, nz->n_int, nz->istart.as<int64_t>(), nz->fid.as<int32_t>(), nz->band.as<double>(),
                lam, cl, static_cast<const double *>(y), static_cast<double *>(z));
    });
    MM_HIP(hipGetLastError());
}

void pair_sum_diff_dev(mm_ctx *ctx, int64_t n, mm_precision prec, const void *a, const void *b,
                       void *plus, void *minus) {
    const int grid = grid_for(n);
    if (prec == MM_F32)
        k_sum_diff<float><<<grid, BS, 0, ctx->stream>>>(
            n, static_cast<const float *>(a), static_cast<const float *>(b),
            static_cast<float *>(plus), static_cast<float *>(minus));
    else
        k_sum_diff<double><<<grid, BS, 0, ctx->stream>>>(
            n, static_cast<const double *>(a), static_cast<const double *>(b),
            static_cast<double *>(plus), static_cast<double *>(minus));
    MM_HIP(hipGetLastError());
}

void mask_tod_dev(mm_ctx *ctx, const mm_pointing *p, int nrhs, const void *tod, void *y,
                  int *flag) {
    const int64_t n = p->n_samp;
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        const int grid = grid_for(n * R);
        if (p->prec == MM_F32)
            k_mask<float, R><<<grid, BS, 0, ctx->stream>>>(p->j.as<int32_t>(), n,
                                                           static_cast<const float *>(tod),
                                                           static_cast<float *>(y), flag);
        else
            k_mask<double, R><<<grid, BS, 0, ctx->stream>>>(p->j.as<int32_t>(), n,
                                                            static_cast<const double *>(tod),
                                                            static_cast<double *>(y), flag);
    });
    MM_HIP(hipGetLastError());
}

}  // namespace mm

namespace mm {

// Tile counts of the direct band for every column count R = 2^li (tile
// length band_tile_len(R)): pref[li][i] = tiles in the intervals before i.
void build_band_tiles(mm_ctx *ctx, mm_noise *nz) {
    const size_t np = (size_t)nz->n_int + 1;
    nz->h_tile_pref.assign(7 * np, 0);
    for (int li = 0; li < 7; ++li) {
        const int64_t tl = band_tile_len(1 << li, nz->band_small);
        int64_t *pr = nz->h_tile_pref.data() + li * np;
        for (int i = 0; i < nz->n_int; ++i)
            pr[i + 1] = pr[i] + (nz->h_istart[i + 1] - nz->h_istart[i] + tl - 1) / tl;
    }
    nz->tile_pref.alloc(sizeof(int64_t) * nz->h_tile_pref.size());
    MM_HIP(hipMemcpyAsync(nz->tile_pref.ptr, nz->h_tile_pref.data(),
                          sizeof(int64_t) * nz->h_tile_pref.size(), hipMemcpyHostToDevice,
                          ctx->stream));
    MM_HIP(hipStreamSynchronize(ctx->stream));
}

// Measure candidates for each stage with HIP events and keep the fastest:
//   stage 0, P: the grid size (grid-stride kernels);
//   stage 1, direct band: the taps per LDS chunk (smaller chunks need less
//     LDS per block, so more blocks share a CU);
//   stage 2, P^T with several columns: visiting the pixels in the tiled
//     order or ascending;
//   stage 3 (flag MM_TUNE_FFT_BLOCK only), FFT: the overlap-save block length.
// Stages 0-2 change speed only: every output sums its terms in a fixed order
// that no candidate changes, so results are bitwise the same.  Stage 3 moves
// results at the rounding level.  report: (stage, candidate, ms) triples.
void autotune(mm_ctx *ctx, mm_pointing *p, mm_noise *nz, int nrhs, int flags, double *report,
              int *n_report, int max_report) {
    const int li = log2i(nrhs);
    const size_t te = p->prec == MM_F32 ? sizeof(float) : sizeof(double);
    DBuf x, y, z;
    x.alloc(sizeof(double) * (size_t)p->n() * nrhs);
    y.alloc(te * (size_t)p->n_samp * nrhs);
    z.alloc(te * (size_t)p->n_samp * nrhs);
    MM_HIP(hipMemsetAsync(x.ptr, 0, x.bytes, ctx->stream));
    MM_HIP(hipMemsetAsync(y.ptr, 0, y.bytes, ctx->stream));
    hipEvent_t e0, e1;
    MM_HIP(hipEventCreate(&e0));
    MM_HIP(hipEventCreate(&e1));
    int nr = 0;
    auto time_it = [&](const std::function<void()> &f) {
        f();
        MM_HIP(hipEventRecord(e0, ctx->stream));
        for (int i = 0; i < 5; ++i) f();
        MM_HIP(hipEventRecord(e1, ctx->stream));
        MM_HIP(hipEventSynchronize(e1));
        float ms = 0;
        MM_HIP(hipEventElapsedTime(&ms, e0, e1));
        return ms / 5.0;
    };
    auto note = [&](int stage, double cand, double ms) {
        if (report && nr < max_report) {
            report[3 * nr] = stage;
            report[3 * nr + 1] = cand;
            report[3 * nr + 2] = ms;
        }
        ++nr;
    };
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    try {
        // stage 0: P grid size
        {
            double best = 1e30;
            int best_g = 0;
            for (int mult : {2, 4, 8, 16, 32}) {
                const int g = ctx->n_cu * mult;
                p->p_blocks[li] = g;
                const double ms =
                    time_it([&]() { apply_P_dev(ctx, p, nrhs, x.as<double>(), y.ptr); });
                note(0, g, ms);
                if (ms < best) { best = ms; best_g = g; }
            }
            p->p_blocks[li] = best_g;
        }
        // stage 1: taps per LDS chunk of the direct band
        if (nz->method == MM_NOISE_DIRECT) {
            const int def = band_chunk(nz->half_bw, nrhs, nz->prec, nz->band_small);
            double best = 1e30;
            int best_c = 0;
            for (int div : {1, 2, 4, 8}) {
                const int c = def / div / BT_OPT * BT_OPT;
                if (c < BT_OPT || (div > 1 && c == def)) continue;
                nz->band_cl[li] = c;
                const double ms = time_it([&]() { noise_apply_dev(ctx, nz, nrhs, y.ptr, z.ptr); });
                note(1, c, ms);
                if (ms < best) { best = ms; best_c = c; }
            }
            nz->band_cl[li] = best_c == def ? 0 : best_c;
        }
        // stage 2: visiting order of the one-wave-per-pixel P^T
        if (nrhs > 1 && p->seg_order.ptr) {
            double best = 1e30;
            int best_o = -1;
            for (int o : {1, 0}) {
                p->pt_order[li] = o;
                const double ms = time_it([&]() { apply_PT_dev(ctx, p, nrhs, z.ptr, x.as<double>()); });
                note(2, o, ms);
                if (ms < best) { best = ms; best_o = o; }
            }
            p->pt_order[li] = best_o;
        }
        // stage 3: FFT block length (results move at the rounding level)
        if ((flags & MM_TUNE_FFT_BLOCK) && nz->method == MM_NOISE_FFT) {
            const int keep = nz->fft_n;
            double best = 1e30;
            int best_n = keep;
            for (int n_fft : {16384, 32768}) {
                if (n_fft == 16384 && nz->half_bw > 6144) continue;
                MM_HIP(hipStreamSynchronize(ctx->stream));
                noise_fft_prepare(ctx, nz, n_fft);
                const double ms = time_it([&]() { noise_apply_dev(ctx, nz, nrhs, y.ptr, z.ptr); });
                note(3, n_fft, ms);
                if (ms < best) { best = ms; best_n = n_fft; }
            }
            if (best_n != nz->fft_n) {
                MM_HIP(hipStreamSynchronize(ctx->stream));
                noise_fft_prepare(ctx, nz, best_n);
            }
        }
    } catch (...) {
        ctx->prof.on = prof;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    MM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof.on = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_report) *n_report = nr < max_report ? nr : max_report;
}

}  // namespace mm
