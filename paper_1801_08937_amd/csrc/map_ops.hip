// Map-domain kernels: M_BD build/apply (Eq. mbd), deterministic column
// reductions, PCG vector updates (Eq. pcg), the skinny dense products of the
// two-level preconditioner (Eq. m2l) and of the Arnoldi process (Alg.
// arnoldi), the FP64 MFMA Gram product used for E = Z^T (A Z), and the small
// on-device Cholesky of E.
//
// All reductions are two-stage with a fixed partition and a fixed tree, so
// results are bitwise repeatable run to run; no floating-point atomics.
#include "mm_internal.h"

namespace mm {

template <typename T> struct Vec2w;
template <> struct Vec2w<float> { using type = float2; };
template <> struct Vec2w<double> { using type = double2; };

namespace {

constexpr int BS = 256;
using d4m = __attribute__((__vector_size__(4 * sizeof(double)))) double;

// ------------------------------------------------------------------ M_BD

__device__ __forceinline__ int64_t find_interval(const int64_t *__restrict__ istart, int n_int,
                                                 int64_t t) {
    int lo = 0, hi = n_int;  // istart[lo] <= t < istart[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (istart[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// One wave per compact pixel: B_j = sum c0 (1,c,s)(1,c,s)^T; lane 0 inverts.
template <typename T>
__global__ void __launch_bounds__(BS) k_mbd_build(const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ perm,
                                                  const typename Vec2w<T>::type *__restrict__ ws,
                                                  const int64_t *__restrict__ istart, int n_int,
                                                  const int32_t *__restrict__ fid,
                                                  const double *__restrict__ band64, int lam,
                                                  int32_t n_obs, double *__restrict__ inv,
                                                  double *__restrict__ blk,
                                                  double *__restrict__ rcond,
                                                  int *__restrict__ n_bad) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (j >= n_obs) return;
    const int32_t a = off[j], b = off[j + 1];
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t i = a + lane; i < b; i += 64) {
        const int64_t t = perm[i];
        const double c0 = band64[(int64_t)fid[find_interval(istart, n_int, t)] * (lam + 1)];
        const auto ww = ws[i];
        const double c = (double)ww.x, sn = (double)ww.y;
        s[0] += c0;
        s[1] += c0 * c;
        s[2] += c0 * sn;
        s[3] += c0 * c * c;
        s[4] += c0 * c * sn;
        s[5] += c0 * sn * sn;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
        for (int q = 0; q < 6; ++q) s[q] += __shfl_xor(s[q], m);
    if (lane != 0) return;
    // Cholesky B = L L^T with positive pivots
    const double b00 = s[0], b01 = s[1], b02 = s[2], b11 = s[3], b12 = s[4], b22 = s[5];
    bool ok = b00 > 0;
    double l00 = ok ? sqrt(b00) : 1, l10 = b01 / l00, l20 = b02 / l00;
    double d1 = b11 - l10 * l10;
    ok = ok && d1 > 0;
    double l11 = d1 > 0 ? sqrt(d1) : 1, l21 = (b12 - l20 * l10) / l11;
    double d2 = b22 - l20 * l20 - l21 * l21;
    ok = ok && d2 > 0;
    double l22 = d2 > 0 ? sqrt(d2) : 1;
    // L^-1 (lower) then B^-1 = L^-T L^-1
    const double m00 = 1 / l00, m11 = 1 / l11, m22 = 1 / l22;
    const double m10 = -l10 * m00 * m11;
    const double m21 = -l21 * m11 * m22;
    const double m20 = -(l20 * m00 + l21 * m10) * m22;
    double i00 = m00 * m00 + m10 * m10 + m20 * m20;
    double i01 = m11 * m10 + m21 * m20;
    double i02 = m22 * m20;
    double i11 = m11 * m11 + m21 * m21;
    double i12 = m22 * m21;
    double i22 = m22 * m22;
    double nb = fmax(fabs(b00) + fabs(b01) + fabs(b02),
                     fmax(fabs(b01) + fabs(b11) + fabs(b12), fabs(b02) + fabs(b12) + fabs(b22)));
    double ni = fmax(fabs(i00) + fabs(i01) + fabs(i02),
                     fmax(fabs(i01) + fabs(i11) + fabs(i12), fabs(i02) + fabs(i12) + fabs(i22)));
    double rc = ok ? 1.0 / (nb * ni) : 0.0;
    if (!(rc >= 1e-12)) {
        atomicAdd(n_bad, 1);
        ok = false;
    }
    rcond[j] = ok ? rc : 0.0;
    double *o = inv + 6 * j;
    o[0] = i00; o[1] = i01; o[2] = i02; o[3] = i11; o[4] = i12; o[5] = i22;
    double *q = blk + 6 * j;
    q[0] = b00; q[1] = b01; q[2] = b02; q[3] = b11; q[4] = b12; q[5] = b22;
}

// I (NC = 1: B_j = sum c0) and QU (NC = 2: B_j = sum c0 (c, s)(c, s)^T)
// blocks; one wave per compact pixel, lane 0 inverts.  inv holds the packed
// symmetric inverse, (00) or (00, 01, 11).
template <typename T, int NC>
__global__ void __launch_bounds__(BS) k_mbd_build_nc(const int32_t *__restrict__ off,
                                                     const int32_t *__restrict__ perm,
                                                     const typename Vec2w<T>::type *__restrict__ ws,
                                                     const int64_t *__restrict__ istart, int n_int,
                                                     const int32_t *__restrict__ fid,
                                                     const double *__restrict__ band64, int lam,
                                                     int32_t n_obs, double *__restrict__ inv,
                                                     double *__restrict__ blk,
                                                     double *__restrict__ rcond,
                                                     int *__restrict__ n_bad) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (j >= n_obs) return;
    const int32_t a = off[j], b = off[j + 1];
    double s[3] = {0, 0, 0};
    for (int32_t i = a + lane; i < b; i += 64) {
        const int64_t t = perm[i];
        const double c0 = band64[(int64_t)fid[find_interval(istart, n_int, t)] * (lam + 1)];
        if constexpr (NC == 1) {
            s[0] += c0;
        } else {
            const auto ww = ws[i];
            const double c = (double)ww.x, sn = (double)ww.y;
            s[0] += c0 * c * c;
            s[1] += c0 * c * sn;
            s[2] += c0 * sn * sn;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] += __shfl_xor(s[q], m);
    if (lane != 0) return;
    bool ok;
    double rc;
    if constexpr (NC == 1) {
        ok = s[0] > 0;
        inv[j] = ok ? 1.0 / s[0] : 0.0;
        blk[j] = s[0];
        rc = ok ? 1.0 : 0.0;
    } else {
        // Cholesky of [[b00, b01], [b01, b11]], then the inverse
        const double b00 = s[0], b01 = s[1], b11 = s[2];
        ok = b00 > 0;
        const double l00 = ok ? sqrt(b00) : 1, l10 = b01 / l00;
        const double d1 = b11 - l10 * l10;
        ok = ok && d1 > 0;
        const double l11 = d1 > 0 ? sqrt(d1) : 1;
        const double m00 = 1 / l00, m11 = 1 / l11, m10 = -l10 * m00 * m11;
        const double i00 = m00 * m00 + m10 * m10, i01 = m11 * m10, i11 = m11 * m11;
        const double nb = fmax(fabs(b00) + fabs(b01), fabs(b01) + fabs(b11));
        const double ni = fmax(fabs(i00) + fabs(i01), fabs(i01) + fabs(i11));
        rc = ok ? 1.0 / (nb * ni) : 0.0;
        double *o = inv + 3 * j;
        o[0] = i00;
        o[1] = i01;
        o[2] = i11;
        double *q = blk + 3 * j;
        q[0] = b00;
        q[1] = b01;
        q[2] = b11;
    }
    if (!(rc >= 1e-12)) {
        atomicAdd(n_bad, 1);
        ok = false;
    }
    rcond[j] = ok ? rc : 0.0;
}

__global__ void k_min_reduce(const double *__restrict__ v, int64_t n, double *__restrict__ out) {
    __shared__ double sm[BS];
    double m = 1e300;
    for (int64_t i = threadIdx.x; i < n; i += BS) m = fmin(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sm[0];
}

// Block-column partial sums: thread (rg, r) accumulates rows rg, rg + 256/R, ...
// of the block's row range; the 256/R row groups are then combined per column by
// a fixed halving tree in LDS.  partial[blk * R + r].
template <int R>
__device__ __forceinline__ void block_col_reduce(double v, double *__restrict__ partial) {
    __shared__ double sm[BS];
    constexpr int NG = BS / R;
    const int r = threadIdx.x % R, rg = threadIdx.x / R;
    sm[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NG / 2; s > 0; s >>= 1) {
        if (rg < s) sm[rg * R + r] += sm[(rg + s) * R + r];
        __syncthreads();
    }
    if (rg == 0) partial[(int64_t)blockIdx.x * R + r] = sm[r];
}

// out = B_j^-1 v per pixel and column; optionally partial sums of
// dot_with . out per column (fused r.z of PCG).
// Packed symmetric NC x NC block times a vector of NC entries (NC = 1, 2).
template <int NC>
__device__ __forceinline__ void sym_mul(const double *__restrict__ m, const double *u,
                                        double *o) {
    if constexpr (NC == 1) {
        o[0] = m[0] * u[0];
    } else {
        o[0] = m[0] * u[0] + m[1] * u[1];
        o[1] = m[1] * u[0] + m[2] * u[1];
    }
}

template <int R, int NC>
__global__ void __launch_bounds__(BS) k_mbd_apply(const double *__restrict__ inv, int32_t n_obs,
                                                  const double *__restrict__ v,
                                                  double *__restrict__ out,
                                                  const double *__restrict__ dot_with,
                                                  double *__restrict__ partial,
                                                  int64_t pix_per_block) {
    constexpr int NG = BS / R;
    const int r = threadIdx.x % R, rg = threadIdx.x / R;
    const int64_t p0 = (int64_t)blockIdx.x * pix_per_block;
    int64_t p1 = p0 + pix_per_block;
    if (p1 > n_obs) p1 = n_obs;
    double acc = 0;
    if constexpr (NC != 3) {
        for (int64_t j = p0 + rg; j < p1; j += NG) {
            const int64_t base = NC * j * R + r;
            double u[NC], o[NC];
#pragma unroll
            for (int a = 0; a < NC; ++a) u[a] = v[base + a * R];
            sym_mul<NC>(inv + (NC * (NC + 1) / 2) * j, u, o);
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                out[base + a * R] = o[a];
                if (dot_with) acc += dot_with[base + a * R] * o[a];
            }
        }
        if (partial) block_col_reduce<R>(acc, partial);
        return;
    }
    for (int64_t j = p0 + rg; j < p1; j += NG) {
        const double *m = inv + 6 * j;
        const int64_t base = 3 * j * R + r;
        const double v0 = v[base], v1 = v[base + R], v2 = v[base + 2 * R];
        const double o0 = m[0] * v0 + m[1] * v1 + m[2] * v2;
        const double o1 = m[1] * v0 + m[3] * v1 + m[4] * v2;
        const double o2 = m[2] * v0 + m[4] * v1 + m[5] * v2;
        out[base] = o0;
        out[base + R] = o1;
        out[base + 2 * R] = o2;
        if (dot_with) acc += dot_with[base] * o0 + dot_with[base + R] * o1 +
                             dot_with[base + 2 * R] * o2;
    }
    if (partial) block_col_reduce<R>(acc, partial);
}

// ------------------------------------------------------------- reductions

template <int R>
__global__ void __launch_bounds__(BS) k_dot_partial(int64_t n, const double *__restrict__ a,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ partial,
                                                    int64_t rows_per_block) {
    constexpr int NG = BS / R;
    const int r = threadIdx.x % R, rg = threadIdx.x / R;
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t i1 = i0 + rows_per_block;
    if (i1 > n) i1 = n;
    double acc = 0;
    for (int64_t i = i0 + rg; i < i1; i += NG) acc += a[i * R + r] * b[i * R + r];
    block_col_reduce<R>(acc, partial);
}

// Second stage: one wave per column sums partial[b * R + r] over b in a fixed
// order (lane-strided, then a xor butterfly).
__device__ __forceinline__ double wave_sum_parts(const double *__restrict__ partial, int n_part,
                                                 int R, int r) {
    const int lane = threadIdx.x & 63;
    double s = 0;
    for (int b = lane; b < n_part; b += 64) s += partial[(int64_t)b * R + r];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    return s;
}

__global__ void k_dot_final(const double *__restrict__ partial, int n_part, int R,
                            double *__restrict__ out) {
    const int r = blockIdx.x;
    const double s = wave_sum_parts(partial, n_part, R, r);
    if ((threadIdx.x & 63) == 0) out[r] = s;
}

// ------------------------------------------------------------------- PCG

__global__ void k_pcg_init(int R, PcgDev s, double tol) {
    const int r = threadIdx.x;
    if (r >= R) return;
    s.done[r] = 0;
    s.brk[r] = 0;
    s.iters[r] = 0;
    s.tol2[r] = tol * tol;
}

// r = b - Ax  (all columns)
template <int R>
__global__ void __launch_bounds__(BS) k_axpby(int64_t n, const double *__restrict__ b,
                                              const double *__restrict__ ax,
                                              double *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n * R;
         e += (int64_t)gridDim.x * BS)
        out[e] = b[e] - ax[e];
}

// Several columns: alpha = rho / p.q in a launch of its own, breakdown if
// p.q <= 0
__global__ void k_pcg_alpha(const double *__restrict__ partial, int n_part, int R, PcgDev s) {
    const int r = blockIdx.x;
    const double pq = wave_sum_parts(partial, n_part, R, r);
    if ((threadIdx.x & 63) != 0) return;
    s.pq[r] = pq;
    if (s.done[r]) return;
    if (!(pq > 0.0)) {
        s.brk[r] = 1;
        s.done[r] = 1;
        s.alpha[r] = 0;
        return;
    }
    s.alpha[r] = s.rho[r] / pq;
}

// x += alpha p; r -= alpha q (live columns); partial ||r||^2.
// One column (pq_part given): alpha = rho / p.q is taken here.  Every block
// sums the p.q partials itself, in the same order, so all take the same
// alpha; block 0 records p.q and alpha.  A column whose p.q is not positive
// (breakdown) is left as it is and flagged by k_pcg_rnrz, so that no block
// reads a flag another block of this launch writes.  Several columns
// (pq_part null): alpha and the flags come from k_pcg_alpha, since 64 such
// sums per block cost more than the launch they save.
template <int R>
__global__ void __launch_bounds__(BS) k_pcg_xr(int64_t n, PcgDev s,
                                               const double *__restrict__ pq_part, int n_part,
                                               const double *__restrict__ p,
                                               const double *__restrict__ q,
                                               double *__restrict__ x, double *__restrict__ rr,
                                               double *__restrict__ partial,
                                               int64_t rows_per_block) {
    constexpr int NG = BS / R;
    const int r = threadIdx.x % R, rg = threadIdx.x / R;
    bool live;
    double al;
    if (R == 1 && pq_part) {
        __shared__ double s_al;
        __shared__ int s_live;
        if (threadIdx.x < 64) {
            const double pq = wave_sum_parts(pq_part, n_part, 1, 0);
            if (threadIdx.x == 0) {
                const bool was_done = s.done[0] != 0;
                const bool lv = !was_done && pq > 0.0;
                const double a = lv ? s.rho[0] / pq : 0.0;
                s_al = a;
                s_live = lv;
                if (blockIdx.x == 0) {
                    s.pq[0] = pq;
                    if (!was_done) s.alpha[0] = a;
                }
            }
        }
        __syncthreads();
        live = s_live != 0;
        al = s_al;
    } else {
        live = !s.done[r];
        al = s.alpha[r];
    }
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t i1 = i0 + rows_per_block;
    if (i1 > n) i1 = n;
    double acc = 0;
    for (int64_t i = i0 + rg; i < i1; i += NG) {
        const int64_t e = i * R + r;
        double rv = rr[e];
        if (live) {
            x[e] += al * p[e];
            rv -= al * q[e];
            rr[e] = rv;
        }
        acc += rv * rv;
    }
    block_col_reduce<R>(acc, partial);
}

// ||r||^2; iteration count and convergence flag
__global__ void k_pcg_rn(const double *__restrict__ partial, int n_part, int R, PcgDev s,
                         int count_iter) {
    const int r = blockIdx.x;
    const double rn = wave_sum_parts(partial, n_part, R, r);
    if ((threadIdx.x & 63) != 0) return;
    if (count_iter) {
        if (s.done[r]) return;
        s.iters[r] += 1;
    }
    s.rn2[r] = rn;
    if (s.hist && s.iters[r] < s.hist_len) s.hist[(int64_t)s.iters[r] * R + r] = rn;
    if (rn <= s.tol2[r] * s.bn2[r]) s.done[r] = 1;
}

// rho' = r.z; beta = rho'/rho (init: rho = r.z, beta unused)
__global__ void k_pcg_rz(const double *__restrict__ partial, int n_part, int R, PcgDev s,
                         int init) {
    const int r = blockIdx.x;
    const double rz = wave_sum_parts(partial, n_part, R, r);
    if ((threadIdx.x & 63) != 0) return;
    if (init) {
        s.rho[r] = rz;
        s.beta[r] = 0;
        return;
    }
    if (s.done[r]) return;
    s.beta[r] = s.rzo ? (rz - s.rzo[r]) / s.rho[r] : rz / s.rho[r];
    s.rho[r] = rz;
}

// The two scalar steps between the x, r update and the p update of one
// iteration, in one launch: a breakdown of this iteration's p.q ends the
// column (its alpha was taken as 0); otherwise ||r||^2 counts the iteration
// and tests convergence; a live column then takes rho' = r.z and
// beta = rho'/rho (Polak-Ribiere with r'.z_old when that is kept).
__global__ void k_pcg_rnrz(const double *__restrict__ part_rn, const double *__restrict__ part_rz,
                           int n_part, int R, PcgDev s) {
    const int r = blockIdx.x;
    const double rn = wave_sum_parts(part_rn, n_part, R, r);
    const double rz = wave_sum_parts(part_rz, n_part, R, r);
    if ((threadIdx.x & 63) != 0) return;
    if (s.done[r]) return;
    if (!(s.pq[r] > 0.0)) {
        s.brk[r] = 1;
        s.done[r] = 1;
        return;
    }
    s.iters[r] += 1;
    s.rn2[r] = rn;
    if (s.hist && s.iters[r] < s.hist_len) s.hist[(int64_t)s.iters[r] * R + r] = rn;
    if (rn <= s.tol2[r] * s.bn2[r]) {
        s.done[r] = 1;
        return;
    }
    s.beta[r] = s.rzo ? (rz - s.rzo[r]) / s.rho[r] : rz / s.rho[r];
    s.rho[r] = rz;
}

__global__ void k_pcg_rzo(const double *__restrict__ partial, int n_part, int R, PcgDev s) {
    const int r = blockIdx.x;
    const double v = wave_sum_parts(partial, n_part, R, r);
    if ((threadIdx.x & 63) == 0) s.rzo[r] = v;
}

template <int R>
__global__ void __launch_bounds__(BS) k_pcg_p(int64_t n, PcgDev s, const double *__restrict__ z,
                                              double *__restrict__ p) {
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n * R;
         e += (int64_t)gridDim.x * BS) {
        const int r = (int)(e % R);
        if (!s.done[r]) p[e] = z[e] + s.beta[r] * p[e];
    }
}

template <int R>
__global__ void __launch_bounds__(BS) k_copy_masked(int64_t n, const int *__restrict__ done,
                                                    const double *__restrict__ src,
                                                    double *__restrict__ dst) {
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < n * R;
         e += (int64_t)gridDim.x * BS) {
        const int r = (int)(e % R);
        if (!done || !done[r]) dst[e] = src[e];
    }
}

// -------------------------------------------------------- skinny products

// partial[chunk * ncol + col] = sum_{i in chunk} W[col * n + i] v[i], one
// column per block (many columns: the Arnoldi basis).
__global__ void __launch_bounds__(BS) k_gemv_t(int64_t n, const double *__restrict__ W,
                                               const double *__restrict__ v,
                                               double *__restrict__ partial, int64_t rows,
                                               int ncol) {
    const int col = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * rows;
    int64_t i1 = i0 + rows;
    if (i1 > n) i1 = n;
    const double *w = W + (int64_t)col * n;
    double acc = 0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BS) acc += w[i] * v[i];
    __shared__ double sm[BS];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * ncol + col] = sm[0];
}

// The same for GT columns at once (col = blockIdx.y GT + c), for few
// columns (Z^T v of M_2l): v is read once
// per group of columns, and each thread keeps GT independent loads in
// flight.  Each column sums a thread's rows in order, then the lanes of a
// wave by a fixed transpose reduction (below), then the waves in order.
constexpr int GT = 16;

// Sums over the 64 lanes of a wave for the 16 values a[0..15] every lane
// holds.  At the exchanges with lanes xor 32, 16, 8 and 4 a lane keeps half
// of its remaining columns (the upper half when that lane bit is set) and
// adds its partner's copy of them, so the columns left halve each time:
// 8 + 4 + 2 + 1 exchanges, then two more (xor 2, xor 1) on the last value,
// instead of six for each of the 16 columns.  Returns the total of column
// (lane >> 2) & 15.  The order of the additions is fixed.
__device__ __forceinline__ double wave_sum16_transposed(double (&a)[16], int lane) {
#pragma unroll
    for (int h = 8, d = 32; h >= 1; h >>= 1, d >>= 1) {
        const bool up = (lane & d) != 0;
#pragma unroll
        for (int c = 0; c < h; ++c) {
            const double send = up ? a[c] : a[c + h];
            const double keep = up ? a[c + h] : a[c];
            a[c] = keep + __shfl_xor(send, d);
        }
    }
    double t = a[0];
    t += __shfl_xor(t, 2);
    t += __shfl_xor(t, 1);
    return t;
}
__global__ void __launch_bounds__(BS) k_gemv_t_grp(int64_t n, const double *__restrict__ W,
                                                   const double *__restrict__ v,
                                                   double *__restrict__ partial, int64_t rows,
                                                   int ncol) {
    const int c0 = blockIdx.y * GT;
    const int nc = ncol - c0 < GT ? ncol - c0 : GT;
    const int64_t i0 = (int64_t)blockIdx.x * rows;
    int64_t i1 = i0 + rows;
    if (i1 > n) i1 = n;
    double acc[GT];
#pragma unroll
    for (int c = 0; c < GT; ++c) acc[c] = 0;
    const double *w = W + (int64_t)c0 * n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BS) {
        const double vi = v[i];
        // every column's load is issued unconditionally (columns past nc
        // re-read the last one and are not accumulated), so the GT loads are
        // in flight together instead of one branch and wait each
        double x[GT];
#pragma unroll
        for (int c = 0; c < GT; ++c) x[c] = w[(int64_t)(c < nc ? c : nc - 1) * n + i];
#pragma unroll
        for (int c = 0; c < GT; ++c) acc[c] = c < nc ? acc[c] + x[c] * vi : acc[c];
    }
    __shared__ double sm[BS / 64][GT];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double tot = wave_sum16_transposed(acc, lane);
    if ((lane & 3) == 0) sm[wv][(lane >> 2) & 15] = tot;
    __syncthreads();
    if (threadIdx.x < nc) {
        double t = 0;
#pragma unroll
        for (int q = 0; q < BS / 64; ++q) t += sm[q][threadIdx.x];
        partial[(int64_t)blockIdx.x * ncol + c0 + threadIdx.x] = t;
    }
}

// v[i] -= sum_c W[c n + i] h[c]
__global__ void __launch_bounds__(BS) k_gemv_n_sub(int64_t n, int ncol,
                                                   const double *__restrict__ W,
                                                   const double *__restrict__ h,
                                                   double *__restrict__ v) {
    __shared__ double sh[512];
    for (int c = threadIdx.x; c < ncol; c += BS) sh[c] = h[c];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        double acc = 0;
        for (int c = 0; c < ncol; ++c) acc += W[(int64_t)c * n + i] * sh[c];
        v[i] -= acc;
    }
}

// dst = src * s or src / s, s a device scalar
__global__ void k_scale(int64_t n, const double *__restrict__ src, const double *__restrict__ s,
                        double *__restrict__ dst, int invert) {
    const double f = invert ? 1.0 / *s : *s;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        dst[i] = src[i] * f;
}

// Zout = V Y for tall V (n x kin, column-major) and small Y (kin x kout,
// column-major, kout <= 64) on FP64 MFMA: each wave owns 16 output rows and
// all kout columns (up to four 16 x 16 accumulators), stepping through kin four
// columns of V at a time.
__global__ void __launch_bounds__(BS) k_gemm_tall_small(int64_t n, int kin, int kout,
                                                        const double *__restrict__ V,
                                                        const double *__restrict__ Y,
                                                        double *__restrict__ Zo) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
    if (row0 >= n) return;
    const int i16 = lane % 16, k4 = lane / 16;
    const int64_t arow = row0 + i16;
    const int TB = (kout + 15) / 16;
    d4m acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4m{0, 0, 0, 0};
    for (int m = 0; m < kin; m += 4) {
        const int mm = m + k4;
        const double av = (arow < n && mm < kin) ? V[(int64_t)mm * n + arow] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < TB) {
                const int col = q * 16 + i16;
                const double bv = (mm < kin && col < kout) ? Y[(int64_t)col * kin + mm] : 0.0;
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
    // item v of lane l holds row l/16 + 4 v, column l % 16
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < TB) {
            const int col = q * 16 + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + k4 + 4 * v;
                if (row < n && col < kout) Zo[(int64_t)col * n + row] = acc[q][v];
            }
        }
    }
}

// --------------------------------------------------------- MFMA Gram (FP64)
//
// C[a][b] = sum_i X(i, a) Y(i, b), X(i, a) = X[i*xr + a*xc], likewise Y.
// Block = 4 waves over the block's rows; wave w owns the 16 x 16 output tiles
// w, w + 4, ..., and walks the rows once per tile.  Each wave loads its
// v_mfma_f64_16x16x4f64 operands straight from global memory (lane l feeds
// row l/16 and column l%16 of the 16 x 4 A and B fragments), GR_KS K-steps
// of 4 rows at a time in flight, with no LDS and no barriers.  Each block writes its partial KA x KB product; a second
// kernel sums the partials in a fixed order.

using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

constexpr int GR_KS = 8;                // K-steps of 4 rows in flight per group
constexpr int GR_ROWS = 4 * GR_KS;      // rows per group

__global__ void __launch_bounds__(BS) k_gram_mfma(int64_t n, int ka, int kb,
                                                  const double *__restrict__ X, int64_t xr,
                                                  int64_t xc, const double *__restrict__ Y,
                                                  int64_t yr, int64_t yc,
                                                  double *__restrict__ partial,
                                                  int64_t rows_per_block) {
    const int KA = (ka + 15) & ~15, KB = (kb + 15) & ~15;  // <= 64 each
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int TA = KA / 16, TB = KB / 16, NT = TA * TB;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t i1 = i0 + rows_per_block;
    if (i1 > n) i1 = n;
    const uint32_t uxr = (uint32_t)xr, uyr = (uint32_t)yr;
    const int64_t P = gridDim.x;
    // the wave's tiles one after another: one accumulator live at a time
    for (int t = wv; t < NT; t += 4) {
        const int ta = t / TB, tb = t % TB;
        const int a = ta * 16 + m, b = tb * 16 + m;
        // this lane's column of A and of B as element offsets (32-bit: the
        // host checks the index range); a padding column feeds 0
        const bool xa = a < ka, yb = b < kb;
        const uint32_t xo = xa ? (uint32_t)(a * xc) : 0u, yo = yb ? (uint32_t)(b * yc) : 0u;
        d4 acc = d4{0, 0, 0, 0};
        for (int64_t rb = i0; rb < i1; rb += GR_ROWS) {
            double av[GR_KS], bv[GR_KS];
#pragma unroll
            for (int s = 0; s < GR_KS; ++s) {
                const int64_t row = rb + 4 * s + kq;
                const bool rok = row < i1;
                const uint32_t ur = (uint32_t)row;
                av[s] = (xa && rok) ? X[ur * uxr + xo] : 0.0;
                bv[s] = (yb && rok) ? Y[ur * uyr + yo] : 0.0;
            }
#pragma unroll
            for (int s = 0; s < GR_KS; ++s)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
        }
        // D layout of v_mfma_f64_16x16x4f64 (checked on gfx950): item v of
        // lane l holds row l/16 + 4 v, column l % 16.  Partials are stored
        // element-major, partial[(row 64 + col) P + block].
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = ta * 16 + (lane / 16) + 4 * v;
            const int col = tb * 16 + (lane % 16);
            partial[(int64_t)(row * 64 + col) * P + blockIdx.x] = acc[v];
        }
    }
}

// One wave per element: lane-strided partial sums over the blocks, then a
// xor butterfly (a fixed order).
__global__ void k_gram_final(const double *__restrict__ partial, int n_part, int ka, int kb,
                             double *__restrict__ C) {
    const int e = (blockIdx.x * BS + threadIdx.x) >> 6, lane = threadIdx.x & 63;
    if (e >= ka * kb) return;
    const int a = e / kb, b = e % kb;
    const double *pp = partial + (int64_t)(a * 64 + b) * n_part;
    double s = 0;
    for (int p = lane; p < n_part; p += 64) s += pp[p];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) C[a * kb + b] = s;
}

// -------------------------------------------------------- small Cholesky
//
// E (k x k row-major, k <= 64) -> symmetrised E_s = (E + E^T)/2 (written back)
// and its lower factor Lc (row-major).  flag = 1 if a pivot^2 falls below
// 1e-13 * max diag (numerically not SPD).
__global__ void k_chol_small(int k, double *__restrict__ E, double *__restrict__ Lc,
                             int *__restrict__ flag) {
    __shared__ double A[64][65];
    const int tid = threadIdx.x;
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        A[i][j] = 0.5 * (E[i * k + j] + E[j * k + i]);
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += blockDim.x) E[e] = A[e / k][e % k];
    __shared__ double dmax;
    __shared__ int bad;
    if (tid == 0) {
        double m = 0;
        for (int i = 0; i < k; ++i) m = fmax(m, A[i][i]);
        dmax = m;
        bad = 0;
    }
    __syncthreads();
    for (int c = 0; c < k; ++c) {
        if (tid == 0) {
            double d = A[c][c];
            if (!(d > 1e-13 * dmax)) { bad = 1; d = 1e-300; }
            A[c][c] = sqrt(d);
        }
        __syncthreads();
        const double lcc = A[c][c];
        for (int i = c + 1 + tid; i < k; i += blockDim.x) A[i][c] /= lcc;
        __syncthreads();
        for (int e = tid; e < (k - c - 1) * (k - c - 1); e += blockDim.x) {
            const int i = c + 1 + e / (k - c - 1), j = c + 1 + e % (k - c - 1);
            if (j <= i) A[i][j] -= A[i][c] * A[j][c];
        }
        __syncthreads();
    }
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        Lc[e] = j <= i ? A[i][j] : 0.0;
    }
    if (tid == 0) *flag = bad;
}

// U[c n + i] += g[c] r[i]: a rank-one update of the column-major n x k U.
__global__ void __launch_bounds__(BS) k_rank1_add(int64_t n, int k, const double *__restrict__ r,
                                                  const double *__restrict__ g,
                                                  double *__restrict__ U) {
    const int64_t tot = n * k;
    for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * BS) {
        const int64_t c = e / n;
        U[e] += g[c] * r[e - c * n];
    }
}

// Lane j's value of v (j uniform across the wave), as two 32-bit reads.
__device__ __forceinline__ double lane_value(double v, int j) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Column r of E^-1 (block r) from the Cholesky factor L of E: forward then
// backward substitution on e_r, column by column.  Lane i holds y_i.  At
// step j, y_j is final: it is read from lane j, scaled by 1 / L_jj (each lane
// forms the reciprocal of its own diagonal entry once), and every lane still
// to be solved subtracts its multiple of it, so each y_i is updated in the
// fixed order of j.  Column r is stored contiguously: Einv[r k + i] =
// (E^-1)_{i r}.  Formed once per M_2l, so that its applies need no
// substitution.
__global__ void __launch_bounds__(64) k_coarse_inverse(int k, const double *__restrict__ Lc,
                                                       double *__restrict__ Einv) {
    __shared__ double L[64][65];
    const int i = threadIdx.x, r = blockIdx.x;
    for (int e = i; e < k * k; e += 64) L[e / k][e % k] = Lc[e];
    __syncthreads();
    const bool on = i < k;
    const double rd = on ? 1.0 / L[i][i] : 0.0;
    double y = i == r ? 1.0 : 0.0;
    for (int j = 0; j < k; ++j) {  // L y' = e_r
        const double yj = lane_value(y, j) * lane_value(rd, j);
        if (i == j) y = yj;
        else if (i > j && on) y = __builtin_fma(-L[i][j], yj, y);
    }
    for (int j = k - 1; j >= 0; --j) {  // L^T c = y'
        const double cj = lane_value(y, j) * lane_value(rd, j);
        if (i == j) y = cj;
        else if (i < j) y = __builtin_fma(-L[j][i], cj, y);
    }
    if (on) Einv[(int64_t)r * k + i] = y;
}

// c = E^-1 g for each column r (block r): lane i forms sum_j (E^-1)_{ij} g_j
// in the order of j, with g staged in LDS and the loads of E^-1 issued
// sixteen at a time.  g[a R + r] and c likewise (k x R).
__global__ void __launch_bounds__(64) k_coarse_apply(int k, int R, const double *__restrict__ Einv,
                                                     const double *__restrict__ g,
                                                     double *__restrict__ c) {
    __shared__ double gs[64];
    const int i = threadIdx.x, r = blockIdx.x;
    if (i < k) gs[i] = g[i * R + r];
    __syncthreads();
    if (i >= k) return;
    double acc = 0.0;
    int j = 0;
    for (; j + 16 <= k; j += 16) {
        double e[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) e[q] = Einv[(int64_t)(j + q) * k + i];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = __builtin_fma(e[q], gs[j + q], acc);
    }
    for (; j < k; ++j) acc = __builtin_fma(Einv[(int64_t)j * k + i], gs[j], acc);
    c[i * R + r] = acc;
}

// out = M_BD (v - AZ c) + Z c per pixel and column (Eq. m2l), with optional
// partial sums of dot_with . out.  Z, AZ are column-major n x k, c is k x R.
// One column with g_part given: each block first forms c = E^-1 Z^T v itself
// from the partial sums of Z^T v (g_part[b k + a], b < g_parts), summing each
// column and then forming E^-1 g exactly as k_dot_final and k_coarse_apply
// do, so every block holds the same c, bitwise that of those two launches.
template <int R, int NC>
__global__ void __launch_bounds__(BS) k_m2l_final(const double *__restrict__ inv, int32_t n_obs,
                                                  int k, int64_t n, const double *__restrict__ Z,
                                                  const double *__restrict__ AZ,
                                                  const double *__restrict__ cc,
                                                  const double *__restrict__ g_part, int g_parts,
                                                  const double *__restrict__ Einv,
                                                  const double *__restrict__ v,
                                                  double *__restrict__ out,
                                                  const double *__restrict__ dot_with,
                                                  double *__restrict__ partial,
                                                  int64_t pix_per_block) {
    constexpr int NG = BS / R;
    __shared__ double sc[64 * 64];
    if (R == 1 && g_part) {
        __shared__ double gs[64];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        // wave wv sums columns wv + 4t, eight at a time with their loads in
        // flight together; each column in the order of wave_sum_parts
        for (int a0 = wv; a0 < k; a0 += 4 * 8) {
            double s8[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) s8[t] = 0;
            for (int b = lane; b < g_parts; b += 64) {
                double x8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int a = a0 + 4 * t;
                    x8[t] = g_part[(int64_t)b * k + (a < k ? a : k - 1)];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) s8[t] += x8[t];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                double sm = s8[t];
#pragma unroll
                for (int m = 32; m >= 1; m >>= 1) sm += __shfl_xor(sm, m);
                const int a = a0 + 4 * t;
                if (lane == 0 && a < k) gs[a] = sm;
            }
        }
        __syncthreads();
        if (threadIdx.x < k) {  // c_i = sum_j (E^-1)_{ij} g_j, in the order of j
            const int i = threadIdx.x;
            double acc = 0.0;
            int j = 0;
            for (; j + 16 <= k; j += 16) {
                double e[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) e[q] = Einv[(int64_t)(j + q) * k + i];
#pragma unroll
                for (int q = 0; q < 16; ++q) acc = __builtin_fma(e[q], gs[j + q], acc);
            }
            for (; j < k; ++j) acc = __builtin_fma(Einv[(int64_t)j * k + i], gs[j], acc);
            sc[i] = acc;
        }
    } else {
        for (int e = threadIdx.x; e < k * R; e += BS) sc[e] = cc[e];
    }
    __syncthreads();
    const int r = threadIdx.x % R, rg = threadIdx.x / R;
    const int64_t p0 = (int64_t)blockIdx.x * pix_per_block;
    int64_t p1 = p0 + pix_per_block;
    if (p1 > n_obs) p1 = n_obs;
    double acc = 0;
    if constexpr (NC != 3) {
        for (int64_t j = p0 + rg; j < p1; j += NG) {
            double u[NC], zc[NC], o[NC];
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                const int64_t row = NC * j + a;
                double s_az = 0, s_z = 0;
                for (int q = 0; q < k; ++q) {
                    const double cq = sc[q * R + r];
                    s_az += AZ[(int64_t)q * n + row] * cq;
                    s_z += Z[(int64_t)q * n + row] * cq;
                }
                u[a] = v[row * R + r] - s_az;
                zc[a] = s_z;
            }
            sym_mul<NC>(inv + (NC * (NC + 1) / 2) * j, u, o);
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                const int64_t e = (NC * j + a) * R + r;
                const double oe = o[a] + zc[a];
                out[e] = oe;
                if (dot_with) acc += dot_with[e] * oe;
            }
        }
        if (partial) block_col_reduce<R>(acc, partial);
        return;
    }
    for (int64_t j = p0 + rg; j < p1; j += NG) {
        // the three rows of pixel j together for each q, so a wave reads
        // whole lines of Z and AZ at once (each sum still runs over q in order)
        double u[3], zc[3], s_az[3] = {0, 0, 0};
        zc[0] = zc[1] = zc[2] = 0;
        int q = 0;
        // eight columns' loads issued before their sums, so that they are in
        // flight together (k = 32: four round trips)
        for (; q + 8 <= k; q += 8) {
            double az8[8][3], z8[8][3];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double *azq = AZ + (int64_t)(q + t) * n + 3 * j;
                const double *zq = Z + (int64_t)(q + t) * n + 3 * j;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    az8[t][a] = azq[a];
                    z8[t][a] = zq[a];
                }
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double cq = sc[(q + t) * R + r];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    s_az[a] += az8[t][a] * cq;
                    zc[a] += z8[t][a] * cq;
                }
            }
        }
        for (; q < k; ++q) {
            const double cq = sc[q * R + r];
            const double *azq = AZ + (int64_t)q * n + 3 * j;
            const double *zq = Z + (int64_t)q * n + 3 * j;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s_az[a] += azq[a] * cq;
                zc[a] += zq[a] * cq;
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = v[(3 * j + a) * R + r] - s_az[a];
        const double *m = inv + 6 * j;
        const double o0 = m[0] * u[0] + m[1] * u[1] + m[2] * u[2] + zc[0];
        const double o1 = m[1] * u[0] + m[3] * u[1] + m[4] * u[2] + zc[1];
        const double o2 = m[2] * u[0] + m[4] * u[1] + m[5] * u[2] + zc[2];
        const int64_t base = 3 * j * R + r;
        out[base] = o0;
        out[base + R] = o1;
        out[base + 2 * R] = o2;
        if (dot_with) acc += dot_with[base] * o0 + dot_with[base + R] * o1 +
                             dot_with[base + 2 * R] * o2;
    }
    if (partial) block_col_reduce<R>(acc, partial);
}

// ------------------------------------------------------------- block CG
//
// Out = beta Out + alpha In S for column-batched In, Out ([n][R], R a power
// of two <= 64) and a small S ([R][R] row-major) on FP64 MFMA.  A block takes
// 64 rows: S and the block's rows of In are staged in LDS with coalesced
// loads, then each wave multiplies its 16 rows by S from LDS.
__global__ void __launch_bounds__(BS) k_gemm_rows_small(int64_t n, int lgR,
                                                        const double *__restrict__ In,
                                                        const double *__restrict__ S,
                                                        double alpha, double beta,
                                                        double *__restrict__ Out) {
    __shared__ double sS[64][65];
    __shared__ double sA[64][65];
    const int R = 1 << lgR;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t brow = (int64_t)blockIdx.x * 64;
    for (int e = tid; e < R * R; e += BS) sS[e >> lgR][e & (R - 1)] = S[e];
    for (int e = tid; e < 64 * R; e += BS) {
        const int r = e >> lgR, c = e & (R - 1);
        sA[r][c] = brow + r < n ? In[(brow + r) * R + c] : 0.0;
    }
    __syncthreads();
    const int64_t row0 = brow + wv * 16;
    if (row0 >= n) return;
    const int i16 = lane % 16, k4 = lane / 16;
    const int TB = (R + 15) / 16;
    d4m acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4m{0, 0, 0, 0};
    for (int m = 0; m < R; m += 4) {
        const int mm = m + k4;
        const double av = mm < R ? sA[wv * 16 + i16][mm] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < TB) {
                const int col = q * 16 + i16;
                const double bv = (mm < R && col < R) ? sS[mm][col] : 0.0;
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < TB) {
            const int col = q * 16 + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + k4 + 4 * v;
                if (row < n && col < R) {
                    const int64_t e = row * R + col;
                    Out[e] = (beta == 0.0 ? 0.0 : beta * Out[e]) + alpha * acc[q][v];
                }
            }
        }
    }
}

// G (R x R) -> U with U^T G U = I on the kept directions.  G is symmetrised
// and scaled to unit diagonal (Gs = D^-1 G D^-1, D = diag(G)^1/2) so that the
// drop test measures linear dependence, not magnitude; Gs = L L^T by Cholesky,
// dropping a direction whose pivot^2 is <= tau (numerically dependent on the
// earlier ones) or whose diagonal is not positive; U = D^-1 L^-T, with zero
// rows and columns for dropped directions.  Row-major.  rank[0] = kept count.
constexpr int CHOL_BS = 1024;  // threads of k_chol_inv_drop: a 32 x 32 grid

__global__ void __launch_bounds__(CHOL_BS) k_chol_inv_drop(int R, const double *__restrict__ G,
                                                           double tau, double *__restrict__ U,
                                                           int *__restrict__ rank) {
    __shared__ double A[64][65];
    __shared__ double X[64][65];
    __shared__ double dsc[64];
    __shared__ int keep[64];
    const int tid = threadIdx.x;
    const int ti = tid >> 5, tj = tid & 31;  // 32 x 32 thread grid
    for (int i = tid; i < R; i += CHOL_BS) {
        const double g = G[i * R + i];
        dsc[i] = g > 1e-300 ? sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int i = ti; i < R; i += 32)
        for (int j = tj; j < R; j += 32) {
            const double s = 0.5 * (G[i * R + j] + G[j * R + i]);
            A[i][j] = (dsc[i] > 0 && dsc[j] > 0) ? s / (dsc[i] * dsc[j]) : 0.0;
            X[i][j] = i == j ? 1.0 : 0.0;
        }
    __syncthreads();
    // Right-looking Cholesky, one barrier per column: in the interval of
    // column c every thread reads the pivot A[c][c], the update of the
    // trailing entries (j > c) uses the unscaled column c divided by the
    // pivot, and column c - 1 is scaled (disjoint entries).
    for (int c = 0; c <= R; ++c) {
        if (c > 0) {
            const int q = c - 1;
            const double d = A[q][q];
            const bool kq = dsc[q] > 0 && d > tau;
            const double l = kq ? sqrt(d) : 0.0;
            for (int i = q + 1 + tid; i < R; i += CHOL_BS) A[i][q] = kq ? A[i][q] / l : 0.0;
            if (tid == 0) {
                keep[q] = kq ? 1 : 0;
                A[q][q] = l;
            }
        }
        if (c < R) {
            const double d = A[c][c];
            if (dsc[c] > 0 && d > tau) {
                const double inv = 1.0 / d;
                for (int i = c + 1 + ti; i < R; i += 32)
                    for (int j = c + 1 + tj; j <= i; j += 32) A[i][j] -= A[i][c] * A[j][c] * inv;
            }
        }
        __syncthreads();
    }
    // X = L^-1 on the kept directions, by row elimination on [L | I]: at step
    // k the rows below k take row k times L[i][k] / L[k][k] (row k is final:
    // only earlier steps change it), and row k - 1 is divided by its pivot
    // (no later step reads it).  A dropped direction has L[k][k] = 0 and a
    // zero column, so its row of X is zeroed and feeds no other row.
    for (int k = 0; k <= R; ++k) {
        if (k > 0) {
            const int q = k - 1;
            const double l = A[q][q];
            for (int j = tid; j < R; j += CHOL_BS) X[q][j] = keep[q] ? X[q][j] / l : 0.0;
        }
        if (k < R && keep[k]) {
            const double inv = 1.0 / A[k][k];
            for (int i = k + 1 + ti; i < R; i += 32) {
                const double f = A[i][k] * inv;
                if (f != 0.0)
                    for (int j = tj; j <= k; j += 32) X[i][j] -= f * X[k][j];
            }
        }
        __syncthreads();
    }
    for (int i = ti; i < R; i += 32)
        for (int j = tj; j < R; j += 32)
            U[i * R + j] = dsc[i] > 0 ? X[j][i] / dsc[i] : 0.0;  // D^-1 (L^-1)^T
    if (tid == 0) {
        int r = 0;
        for (int c = 0; c < R; ++c) r += keep[c];
        rank[0] = r;
    }
}

// ----------------------------------------------------- session slot helpers

// dst[i R + slot] = src ? src[i] : 0
__global__ void k_col_set(int64_t n, int R, int slot, const double *__restrict__ src,
                          double *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        dst[i * R + slot] = src ? src[i] : 0.0;
}

// dst[i] = src[i R + slot]
__global__ void k_col_get(int64_t n, int R, int slot, const double *__restrict__ src,
                          double *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        dst[i] = src[i * R + slot];
}

// Rows of a k-column basis moved between two pixel sets by global pixel id:
// dst[c (n_dst) + nc j + a] = src[c n_src + nc i + a] where obs_src[i] =
// obs_dst[j] (binary search; both id lists ascending), 0 when the source set
// lacks the pixel.  One thread per target pixel.
__global__ void __launch_bounds__(BS) k_transfer_rows(int32_t n_dst_obs,
                                                      const int32_t *__restrict__ obs_dst,
                                                      int32_t n_src_obs,
                                                      const int32_t *__restrict__ obs_src,
                                                      int nc, int k, const double *__restrict__ src,
                                                      double *__restrict__ dst) {
    const int32_t j = (int32_t)(blockIdx.x * BS + threadIdx.x);
    if (j >= n_dst_obs) return;
    const int32_t g = obs_dst[j];
    int32_t lo = 0, hi = n_src_obs;  // first index with obs_src[i] >= g
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (obs_src[mid] < g) lo = mid + 1; else hi = mid;
    }
    const bool found = lo < n_src_obs && obs_src[lo] == g;
    const int64_t n_src = (int64_t)nc * n_src_obs, n_dst = (int64_t)nc * n_dst_obs;
    for (int c = 0; c < k; ++c)
        for (int a = 0; a < nc; ++a)
            dst[c * n_dst + (int64_t)nc * j + a] =
                found ? src[c * n_src + (int64_t)nc * lo + a] : 0.0;
}

// mode 0: slot becomes free/stopped (done = 1); mode 1: (re)start with
// tolerance tol (rn2 = bn2, already written), done if already converged.
__global__ void k_slot_ctl(PcgDev s, int slot, int mode, double tol) {
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        s.done[slot] = 1;
        return;
    }
    s.tol2[slot] = tol * tol;
    s.iters[slot] = 0;
    s.brk[slot] = 0;
    s.rn2[slot] = s.bn2[slot];
    s.done[slot] = (s.rn2[slot] <= s.tol2[slot] * s.bn2[slot]) ? 1 : 0;
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

int grid_for(int64_t n, int max_blocks = 4096) {
    int64_t g = (n + BS - 1) / BS;
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

// ----------------------------------------------------------------- launchers

int reduction_parts(int64_t n_rows, int nrhs) {
    const int64_t m = n_rows * nrhs;
    // up to 65,536 elements a block per 256 (one per thread), so that these
    // latency-bound launches spread over more CUs; beyond, a block per 1,024,
    // at most 512 blocks
    int64_t p = m <= 65536 ? (m + 255) / 256 : (m + 1023) / 1024;
    if (p > 512) p = 512;
    return (int)(p < 1 ? 1 : p);
}

static int64_t rows_per(int64_t n, int parts) { return (n + parts - 1) / parts; }

void mbd_build_dev(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz, mm_precond *M,
                   int *n_bad_out) {
    hipStream_t s = ctx->stream;
    const int32_t n_obs = p->n_obs;
    M->inv.alloc(sizeof(double) * packed_sym(p->nc) * (n_obs > 0 ? n_obs : 1));
    M->blk.alloc(sizeof(double) * packed_sym(p->nc) * (n_obs > 0 ? n_obs : 1));
    DBuf rc, bad, mn;
    rc.alloc(sizeof(double) * (n_obs > 0 ? n_obs : 1));
    bad.alloc(sizeof(int));
    mn.alloc(sizeof(double));
    MM_HIP(hipMemsetAsync(bad.ptr, 0, sizeof(int), s));
    if (n_obs > 0) {
        const unsigned nb = (unsigned)((n_obs + 3) / 4);
        auto nc_build = [&](auto TT, auto NN) {
            using T = decltype(TT);
            constexpr int NC = decltype(NN)::value;
            k_mbd_build_nc<T, NC><<<nb, BS, 0, s>>>(
                p->off.as<int32_t>(), p->perm.as<int32_t>(),
                NC == 2 ? static_cast<const typename Vec2w<T>::type *>(p->ws.ptr) : nullptr,
                nz->istart.as<int64_t>(), nz->n_int, nz->fid.as<int32_t>(),
                nz->band64.as<double>(), nz->half_bw, n_obs, M->inv.as<double>(),
                M->blk.as<double>(), rc.as<double>(), bad.as<int>());
        };
        if (p->nc == 1)
            nc_build(0.0, std::integral_constant<int, 1>());
        else if (p->nc == 2 && p->prec == MM_F32)
            nc_build(0.f, std::integral_constant<int, 2>());
        else if (p->nc == 2)
            nc_build(0.0, std::integral_constant<int, 2>());
        else if (p->prec == MM_F32)
            k_mbd_build<float><<<nb, BS, 0, s>>>(p->off.as<int32_t>(), p->perm.as<int32_t>(),
                                                 p->ws.as<float2>(), nz->istart.as<int64_t>(),
                                                 nz->n_int, nz->fid.as<int32_t>(),
                                                 nz->band64.as<double>(), nz->half_bw, n_obs,
                                                 M->inv.as<double>(), M->blk.as<double>(),
                                                 rc.as<double>(), bad.as<int>());
        else
            k_mbd_build<double><<<nb, BS, 0, s>>>(p->off.as<int32_t>(), p->perm.as<int32_t>(),
                                                  p->ws.as<double2>(), nz->istart.as<int64_t>(),
                                                  nz->n_int, nz->fid.as<int32_t>(),
                                                  nz->band64.as<double>(), nz->half_bw, n_obs,
                                                  M->inv.as<double>(), M->blk.as<double>(),
                                                  rc.as<double>(), bad.as<int>());
        k_min_reduce<<<1, BS, 0, s>>>(rc.as<double>(), n_obs, mn.as<double>());
        MM_HIP(hipGetLastError());
    }
    int hb = 0;
    double hm = 1.0;
    MM_HIP(hipMemcpyAsync(&hb, bad.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    if (n_obs > 0) MM_HIP(hipMemcpyAsync(&hm, mn.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    M->rcond_min = hm;
    *n_bad_out = hb;
}

void mbd_apply_dev(mm_ctx *ctx, const double *inv, int32_t n_obs, int nc, int nrhs,
                   const double *v, double *out, const double *dot_with, double *partial,
                   int n_part) {
    Scope sc(ctx->prof, ctx->stream, "precond");
    if (n_obs == 0) return;
    // partition: n_part blocks over pixels (nc rows each)
    const int parts = partial ? n_part : reduction_parts((int64_t)nc * n_obs, nrhs);
    const int64_t ppb = rows_per(n_obs, parts);
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        if (nc == 1)
            k_mbd_apply<R, 1><<<parts, BS, 0, ctx->stream>>>(inv, n_obs, v, out, dot_with,
                                                              partial, ppb);
        else if (nc == 2)
            k_mbd_apply<R, 2><<<parts, BS, 0, ctx->stream>>>(inv, n_obs, v, out, dot_with,
                                                              partial, ppb);
        else
            k_mbd_apply<R, 3><<<parts, BS, 0, ctx->stream>>>(inv, n_obs, v, out, dot_with,
                                                              partial, ppb);
    });
    MM_HIP(hipGetLastError());
}

void dot_partial_cols(mm_ctx *ctx, int64_t n, int nrhs, const double *a, const double *b,
                      double *partial, int n_part) {
    const int64_t rpb = rows_per(n, n_part);
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        k_dot_partial<R><<<n_part, BS, 0, ctx->stream>>>(n, a, b, partial, rpb);
    });
    MM_HIP(hipGetLastError());
}

void dot_cols(mm_ctx *ctx, int64_t n, int nrhs, const double *a, const double *b, double *out) {
    Scope sc(ctx->prof, ctx->stream, "vec");
    const int parts = reduction_parts(n, nrhs);
    ws_alloc(ctx, ctx->red, sizeof(double) * parts * 64);
    dot_partial_cols(ctx, n, nrhs, a, b, ctx->red.as<double>(), parts);
    k_dot_final<<<nrhs, 64, 0, ctx->stream>>>(ctx->red.as<double>(), parts, nrhs, out);
    MM_HIP(hipGetLastError());
}

void pcg_init_scalars(mm_ctx *ctx, int nrhs, PcgDev s, double tol) {
    k_pcg_init<<<1, 64, 0, ctx->stream>>>(nrhs, s, tol);
    MM_HIP(hipGetLastError());
}

void axpby_cols(mm_ctx *ctx, int64_t n, int nrhs, const double *b, const double *Ax, double *r) {
    Scope sc(ctx->prof, ctx->stream, "vec");
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        k_axpby<R><<<grid_for(n * R), BS, 0, ctx->stream>>>(n, b, Ax, r);
    });
    MM_HIP(hipGetLastError());
}

void pcg_after_rnrz(mm_ctx *ctx, int nrhs, PcgDev s, const double *part_rn,
                    const double *part_rz, int n_part) {
    k_pcg_rnrz<<<nrhs, 64, 0, ctx->stream>>>(part_rn, part_rz, n_part, nrhs, s);
    MM_HIP(hipGetLastError());
}

void pcg_update_xr(mm_ctx *ctx, int64_t n, int nrhs, PcgDev s, const double *pq_part,
                   const double *p, const double *q, double *x, double *r, double *partial,
                   int n_part) {
    Scope sc(ctx->prof, ctx->stream, "vec");
    const int64_t rpb = rows_per(n, n_part);
    if (nrhs > 1) {
        k_pcg_alpha<<<nrhs, 64, 0, ctx->stream>>>(pq_part, n_part, nrhs, s);
        MM_HIP(hipGetLastError());
    }
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        k_pcg_xr<R><<<n_part, BS, 0, ctx->stream>>>(n, s, nrhs == 1 ? pq_part : nullptr, n_part,
                                                    p, q, x, r, partial, rpb);
    });
    MM_HIP(hipGetLastError());
}

void pcg_after_rn(mm_ctx *ctx, int nrhs, PcgDev s, const double *partial, int n_part,
                  int count_iter) {
    k_pcg_rn<<<nrhs, 64, 0, ctx->stream>>>(partial, n_part, nrhs, s, count_iter);
    MM_HIP(hipGetLastError());
}

void pcg_after_rz(mm_ctx *ctx, int nrhs, PcgDev s, const double *partial, int n_part, int init) {
    k_pcg_rz<<<nrhs, 64, 0, ctx->stream>>>(partial, n_part, nrhs, s, init);
    MM_HIP(hipGetLastError());
}

void pcg_store_rzo(mm_ctx *ctx, int nrhs, PcgDev s, const double *partial, int n_part) {
    k_pcg_rzo<<<nrhs, 64, 0, ctx->stream>>>(partial, n_part, nrhs, s);
    MM_HIP(hipGetLastError());
}

void pcg_update_p(mm_ctx *ctx, int64_t n, int nrhs, PcgDev s, const double *z, double *p) {
    Scope sc(ctx->prof, ctx->stream, "vec");
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        k_pcg_p<R><<<grid_for(n * R), BS, 0, ctx->stream>>>(n, s, z, p);
    });
    MM_HIP(hipGetLastError());
}

void copy_cols_masked(mm_ctx *ctx, int64_t n, int nrhs, const int *done, const double *src,
                      double *dst) {
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        k_copy_masked<R><<<grid_for(n * R), BS, 0, ctx->stream>>>(n, done, src, dst);
    });
    MM_HIP(hipGetLastError());
}

void gemm_rows_small(mm_ctx *ctx, int64_t n, int R, const double *In, const double *S,
                     double alpha, double beta, double *Out) {
    Scope sc(ctx->prof, ctx->stream, "gemm_mfma");
    MM_CHECK(pow2_ok(R), MM_E_INVALID, "gemm_rows_small: R must be a power of two <= 64");
    k_gemm_rows_small<<<(unsigned)((n + 63) / 64), BS, 0, ctx->stream>>>(n, log2i(R), In, S, alpha,
                                                                      beta, Out);
    MM_HIP(hipGetLastError());
}

void chol_inv_drop(mm_ctx *ctx, int R, const double *G, double tau, double *U, int *rank) {
    k_chol_inv_drop<<<1, CHOL_BS, 0, ctx->stream>>>(R, G, tau, U, rank);
    MM_HIP(hipGetLastError());
}

void col_set(mm_ctx *ctx, int64_t n, int R, int slot, const double *src, double *dst) {
    k_col_set<<<grid_for(n), BS, 0, ctx->stream>>>(n, R, slot, src, dst);
    MM_HIP(hipGetLastError());
}

void transfer_rows(mm_ctx *ctx, int32_t n_dst_obs, const int32_t *obs_dst, int32_t n_src_obs,
                   const int32_t *obs_src, int nc, int k, const double *src, double *dst) {
    if (n_dst_obs <= 0) return;
    k_transfer_rows<<<(n_dst_obs + BS - 1) / BS, BS, 0, ctx->stream>>>(n_dst_obs, obs_dst, n_src_obs,
                                                                       obs_src, nc, k, src, dst);
    MM_HIP(hipGetLastError());
}

void col_get(mm_ctx *ctx, int64_t n, int R, int slot, const double *src, double *dst) {
    k_col_get<<<grid_for(n), BS, 0, ctx->stream>>>(n, R, slot, src, dst);
    MM_HIP(hipGetLastError());
}

void slot_ctl(mm_ctx *ctx, PcgDev s, int slot, int mode, double tol) {
    k_slot_ctl<<<1, 64, 0, ctx->stream>>>(s, slot, mode, tol);
    MM_HIP(hipGetLastError());
}

// The partial sums of W^T v, ctx->red[b ncol + col] for b < the returned
// count of row chunks.
static int gemv_t_parts(mm_ctx *ctx, int64_t n, int ncol, const double *W, const double *v) {
    const int parts = reduction_parts(n);
    ws_alloc(ctx, ctx->red, sizeof(double) * parts * (ncol > 64 ? ncol : 64));
    // grouped columns measured faster for k = 32 (M_2l), one column per
    // block for the long Arnoldi bases
    if (ncol <= 32)
        k_gemv_t_grp<<<dim3(parts, (ncol + GT - 1) / GT), BS, 0, ctx->stream>>>(
            n, W, v, ctx->red.as<double>(), rows_per(n, parts), ncol);
    else
        k_gemv_t<<<dim3(parts, ncol), BS, 0, ctx->stream>>>(n, W, v, ctx->red.as<double>(),
                                                             rows_per(n, parts), ncol);
    MM_HIP(hipGetLastError());
    return parts;
}

void gemv_t(mm_ctx *ctx, int64_t n, int ncol, const double *W, const double *v, double *h) {
    Scope sc(ctx->prof, ctx->stream, "gemv");
    const int parts = gemv_t_parts(ctx, n, ncol, W, v);
    k_dot_final<<<ncol, 64, 0, ctx->stream>>>(ctx->red.as<double>(), parts, ncol, h);
    MM_HIP(hipGetLastError());
}

void gemv_n_sub(mm_ctx *ctx, int64_t n, int ncol, const double *W, const double *h, double *v) {
    Scope sc(ctx->prof, ctx->stream, "gemv");
    MM_CHECK(ncol <= 512, MM_E_INVALID, "gemv: too many columns");
    k_gemv_n_sub<<<grid_for(n, 2048), BS, 0, ctx->stream>>>(n, ncol, W, h, v);
    MM_HIP(hipGetLastError());
}

void rank1_add(mm_ctx *ctx, int64_t n, int k, const double *r, const double *g, double *U) {
    k_rank1_add<<<grid_for(n * k), BS, 0, ctx->stream>>>(n, k, r, g, U);
    MM_HIP(hipGetLastError());
}

void scale_copy(mm_ctx *ctx, int64_t n, const double *src, const double *s_dev, double *dst,
                int invert) {
    k_scale<<<grid_for(n), BS, 0, ctx->stream>>>(n, src, s_dev, dst, invert);
    MM_HIP(hipGetLastError());
}

void matmul_small_right(mm_ctx *ctx, int64_t n, int kin, int kout, const double *V,
                        const double *Y, double *Zo) {
    Scope sc(ctx->prof, ctx->stream, "gemm_mfma");
    MM_CHECK(kout >= 1 && kout <= 64 && kin >= 1, MM_E_INVALID, "matmul_small_right: sizes");
    const int64_t blocks = (n + 63) / 64;
    k_gemm_tall_small<<<(unsigned)blocks, BS, 0, ctx->stream>>>(n, kin, kout, V, Y, Zo);
    MM_HIP(hipGetLastError());
}

void gram_mfma(mm_ctx *ctx, int64_t n, int ka, int kb, const double *X, int64_t x_rs,
               int64_t x_cs, const double *Y, int64_t y_rs, int64_t y_cs, double *C) {
    Scope sc(ctx->prof, ctx->stream, "gram_mfma");
    MM_CHECK(ka >= 1 && ka <= 64 && kb >= 1 && kb <= 64, MM_E_INVALID, "gram: sizes");
    // the kernel indexes with 32-bit element offsets
    MM_CHECK(n >= 1 && x_rs >= 0 && x_cs >= 0 && y_rs >= 0 && y_cs >= 0 &&
                 (n - 1) * x_rs + (int64_t)(ka - 1) * x_cs < ((int64_t)1 << 32) &&
                 (n - 1) * y_rs + (int64_t)(kb - 1) * y_cs < ((int64_t)1 << 32),
             MM_E_INVALID, "gram: operands beyond 2^32 elements");
    // one 32-row chunk per block up to 1,024 blocks (small n: more blocks in
    // flight), then more chunks per block
    int64_t parts64 = (n + GR_ROWS - 1) / GR_ROWS;
    if (parts64 > 1024) parts64 = 1024;
    if (parts64 < 1) parts64 = 1;
    const int parts = (int)parts64;
    int64_t rpb = (n + parts - 1) / parts;
    rpb = (rpb + GR_ROWS - 1) / GR_ROWS * GR_ROWS;
    ws_alloc(ctx, ctx->gram_part, sizeof(double) * 4096 * parts);
    k_gram_mfma<<<parts, BS, 0, ctx->stream>>>(n, ka, kb, X, x_rs, x_cs, Y, y_rs, y_cs,
                                                ctx->gram_part.as<double>(), rpb);
    k_gram_final<<<(ka * kb * 64 + BS - 1) / BS, BS, 0, ctx->stream>>>(
        ctx->gram_part.as<double>(), parts, ka, kb, C);
    MM_HIP(hipGetLastError());
}

void chol_small_dev(mm_ctx *ctx, int k, double *E, double *Lc, int *flag) {
    k_chol_small<<<1, 64, 0, ctx->stream>>>(k, E, Lc, flag);
    MM_HIP(hipGetLastError());
}

void coarse_inverse_dev(mm_ctx *ctx, int k, const double *Lc, double *Einv) {
    k_coarse_inverse<<<k, 64, 0, ctx->stream>>>(k, Lc, Einv);
    MM_HIP(hipGetLastError());
}

void m2l_coef_dev(mm_ctx *ctx, const mm_precond *M, int nrhs, const double *v, double *c) {
    const int64_t n = M->n();
    const int k = M->k;
    ws_alloc(ctx, ctx->coef_g, sizeof(double) * 64 * 64);
    double *g = ctx->coef_g.as<double>();
    if (nrhs == 1) {
        gemv_t(ctx, n, k, M->Z.as<double>(), v, g);
    } else {
        // g[a][r] = sum_i Z[a n + i] v[i R + r]   (Z^T V on MFMA)
        gram_mfma(ctx, n, k, nrhs, M->Z.as<double>(), 1, n, v, nrhs, 1, g);
    }
    k_coarse_apply<<<nrhs, 64, 0, ctx->stream>>>(k, nrhs, M->Einv.as<double>(), g, c);
    MM_HIP(hipGetLastError());
}

void m2l_apply_dev(mm_ctx *ctx, const mm_precond *M, int nrhs, const double *v, double *out,
                   double *partial, int n_part) {
    Scope sc(ctx->prof, ctx->stream, "precond");
    const int64_t n = M->n();
    const int k = M->k;
    ws_alloc(ctx, ctx->scal, sizeof(double) * 64 * 64 + 4096);
    double *c = ctx->scal.as<double>();
    // one column: the Z^T v partial sums go straight to the final kernel,
    // whose blocks each form c = E^-1 Z^T v (two launches fewer)
    const double *g_part = nullptr;
    int g_parts = 0;
    if (nrhs == 1) {
        Scope sg(ctx->prof, ctx->stream, "gemv");
        g_parts = gemv_t_parts(ctx, n, k, M->Z.as<double>(), v);
        g_part = ctx->red.as<double>();
    } else {
        m2l_coef_dev(ctx, M, nrhs, v, c);
    }
    const int parts = partial ? n_part : reduction_parts(n, nrhs);
    const int64_t ppb = rows_per(M->n_obs, parts);
    dispatch_r(nrhs, [&](auto RR) {
        constexpr int R = decltype(RR)::value;
        auto go = [&](auto NN) {
            constexpr int NC = decltype(NN)::value;
            k_m2l_final<R, NC><<<parts, BS, 0, ctx->stream>>>(
                M->inv.as<double>(), M->n_obs, k, n, M->Z.as<double>(), M->AZ.as<double>(), c,
                g_part, g_parts, M->Einv.as<double>(), v, out, partial ? v : nullptr, partial,
                ppb);
        };
        if (M->nc == 1) go(std::integral_constant<int, 1>());
        else if (M->nc == 2) go(std::integral_constant<int, 2>());
        else go(std::integral_constant<int, 3>());
    });
    MM_HIP(hipGetLastError());
}

}  // namespace mm
