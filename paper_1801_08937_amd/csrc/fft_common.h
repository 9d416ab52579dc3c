// Device helpers shared by the FFT kernels of N^-1: 16th roots of unity and
// an in-register radix-2 DFT of 2..16 points.
#pragma once

#include "mm_internal.h"

namespace mm {
namespace fft {

// e^{2 pi i m / 16}
__device__ constexpr double C16[16] = {
    1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898,
    0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867,
    -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898,
    0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867};
__device__ constexpr double S16[16] = {
    0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867,
    1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898,
    0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867,
    -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};

constexpr int ilog2(int r) { return r <= 1 ? 0 : 1 + ilog2(r / 2); }
constexpr int bitrev(int i, int bits) {
    int o = 0;
    for (int b = 0; b < bits; ++b) o |= ((i >> b) & 1) << (bits - 1 - b);
    return o;
}

// In-register R-point DFT, DIR = -1 forward, +1 inverse (radix-2, decimation
// in time).
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_small(T (&re)[R], T (&im)[R]) {
    constexpr int B = ilog2(R);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bitrev(i, B);
        if (i < j) {
            T t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= R; len *= 2) {
        const int half = len / 2;
        const int step = 16 / len;
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int k = 0; k < half; ++k) {
                const T wr = (T)C16[k * step];
                const T wi = (T)(DIR * S16[k * step]);
                const T xr = re[i + k + half], xi = im[i + k + half];
                const T tr = wr * xr - wi * xi;
                const T ti = wr * xi + wi * xr;
                re[i + k + half] = re[i + k] - tr;
                im[i + k + half] = im[i + k] - ti;
                re[i + k] += tr;
                im[i + k] += ti;
            }
        }
    }
}

// 4-point DFT in place, DIR = -1 forward (W4 = -i), +1 inverse.
template <typename T, int DIR>
__device__ __forceinline__ void dft4(T &r0, T &i0, T &r1, T &i1, T &r2, T &i2, T &r3, T &i3) {
    const T ar = r0 + r2, ai = i0 + i2, br = r0 - r2, bi = i0 - i2;
    const T cr = r1 + r3, ci = i1 + i3, dr = r1 - r3, di = i1 - i3;
    // (DIR i) (dr + i di) = DIR (-di + i dr)
    const T er = DIR * -di, ei = DIR * dr;
    r0 = ar + cr; i0 = ai + ci;
    r2 = ar - cr; i2 = ai - ci;
    r1 = br + er; i1 = bi + ei;
    r3 = br - er; i3 = bi - ei;
}

// 16-point DFT as 4 x 4: n = n1 + 4 n2, k = 4 k1 + k2.  Radix-4 over n2,
// twiddle W16^(n1 k2), radix-4 over n1; X[4 k1 + k2] lands in slot k1 + 4 k2
// and is moved to slot 4 k1 + k2 by renaming.
template <typename T, int DIR>
__device__ __forceinline__ void dft16(T (&re)[16], T (&im)[16]) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1)
        dft4<T, DIR>(re[n1], im[n1], re[n1 + 4], im[n1 + 4], re[n1 + 8], im[n1 + 8], re[n1 + 12],
                     im[n1 + 12]);
#pragma unroll
    for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
        for (int k2 = 1; k2 < 4; ++k2) {
            const int m = (n1 * k2) & 15;
            const T wr = (T)C16[m], wi = (T)(DIR * S16[m]);
            const T xr = re[n1 + 4 * k2], xi = im[n1 + 4 * k2];
            re[n1 + 4 * k2] = wr * xr - wi * xi;
            im[n1 + 4 * k2] = wr * xi + wi * xr;
        }
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2)
        dft4<T, DIR>(re[4 * k2], im[4 * k2], re[4 * k2 + 1], im[4 * k2 + 1], re[4 * k2 + 2],
                     im[4 * k2 + 2], re[4 * k2 + 3], im[4 * k2 + 3]);
    // slot k1 + 4 k2 -> 4 k1 + k2 (transpose of the 4 x 4 index grid)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) {
            T t = re[a + 4 * b]; re[a + 4 * b] = re[b + 4 * a]; re[b + 4 * a] = t;
            t = im[a + 4 * b]; im[a + 4 * b] = im[b + 4 * a]; im[b + 4 * a] = t;
        }
}

}  // namespace fft
}  // namespace mm
