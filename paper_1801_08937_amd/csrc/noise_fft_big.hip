// N^-1 by FFT with large overlap-save blocks: N = 32,768 real samples per
// block, packed as NC = 16,384 complex points (same packed-real scheme as
// noise_fft.hip), V = N - 2 lambda valid outputs.  At lambda = 4,096 three
// quarters of every block are valid (half with the 16,384-sample blocks), and
// bandwidths up to 12,288 fit.
//
// 1024 threads each hold 16 complex values in registers through the whole
// transform: radices 16 x 16 x 16 x 4.  Between passes the values are
// exchanged through LDS one component at a time (real parts, then imaginary
// parts), so the exchange buffer is 16,384 FP64 values (xor-swizzled) and the
// thread's other component stays in registers.  The first forward pass reads
// global memory, the radix-4 passes run in registers, the spectrum step reads
// each value's partner Z_{NC-k} through the same LDS buffer, and the last
// inverse pass writes global memory.
#include <cmath>

#include "fft_common.h"

namespace mm {
namespace {

using fft::dft4;
using fft::dft16;

constexpr int BNC = 16384;
constexpr int BN = 2 * BNC;
constexpr int BTH = 1024;
constexpr int BLDS = BNC;
constexpr int BIG_MAX_LAMBDA = 12288;

// LDS index of element i: its low four bits xor-ed with the next four, a
// bijection on [0, BNC) that spreads the stride-16 accesses of the radix-16
// passes over distinct banks without padding.
__device__ __forceinline__ int padb(int i) { return i ^ ((i >> 4) & 15); }

// v[r] *= w1^r, r = 1..R-1, by repeated multiplication.
template <typename T, int R>
__device__ __forceinline__ void twiddle_seq(T (&re)[R], T (&im)[R], T w1r, T w1i) {
    T wr = w1r, wi = w1i;
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const T xr = re[r], xi = im[r];
        re[r] = wr * xr - wi * xi;
        im[r] = wr * xi + wi * xr;
        const T nr = wr * w1r - wi * w1i;
        wi = wr * w1i + wi * w1r;
        wr = nr;
    }
}

// Store component v (value r at LDS index out(r)), then load v[q] from
// index tid + 1024 q.
template <typename T, typename F>
__device__ __forceinline__ void exchange(T *__restrict__ sh, T (&v)[16], const F &out, int tid) {
#pragma unroll
    for (int r = 0; r < 16; ++r) sh[padb(out(r, tid))] = v[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = sh[padb(tid + BTH * q)];
    __syncthreads();
}

// Radix-16 pass at sub-transform size NS on the thread's butterfly j = tid,
// whose inputs x[j + 1024 r] are the registers; twiddle then DFT, leaving the
// outputs for index (j/NS) NS 16 + j mod NS + r NS.
template <typename T, int NS, int DIR>
__device__ __forceinline__ void r16(T (&re)[16], T (&im)[16],
                                    const typename Vec2T<T>::type *__restrict__ tw, int tid) {
    if (NS > 1) {
        const int jm = tid % NS;
        const auto w = tw[jm * (BNC / (NS * 16))];
        twiddle_seq<T, 16>(re, im, w.x, DIR < 0 ? w.y : -w.y);
    }
    dft16<T, DIR>(re, im);
}

template <int NS> struct R16Out {
    __device__ __forceinline__ int operator()(int r, int j) const {
        return (j / NS) * NS * 16 + (j % NS) + r * NS;
    }
};

// Radix-4 pass at NS = 4096, entirely in registers: butterfly jj = tid + 1024 p
// takes x[jj + 4096 r] = register p + 4 r and writes it back in place.
template <typename T, int DIR>
__device__ __forceinline__ void r4_last(T (&re)[16], T (&im)[16],
                                        const typename Vec2T<T>::type *__restrict__ tw, int tid) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int jj = tid + BTH * p;
        T vr[4], vi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            vr[r] = re[p + 4 * r];
            vi[r] = im[p + 4 * r];
        }
        const auto w = tw[jj];
        twiddle_seq<T, 4>(vr, vi, w.x, DIR < 0 ? w.y : -w.y);
        dft4<T, DIR>(vr[0], vi[0], vr[1], vi[1], vr[2], vi[2], vr[3], vi[3]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            re[p + 4 * r] = vr[r];
            im[p + 4 * r] = vi[r];
        }
    }
}

template <typename T, int DIR>
__device__ __forceinline__ void passes_234(T *__restrict__ sh, T (&re)[16], T (&im)[16],
                                           const typename Vec2T<T>::type *__restrict__ tw,
                                           int tid) {
    // after pass 1 the registers hold outputs for index tid*16 + r
    exchange(sh, re, R16Out<1>(), tid);
    exchange(sh, im, R16Out<1>(), tid);
    r16<T, 16, DIR>(re, im, tw, tid);
    exchange(sh, re, R16Out<16>(), tid);
    exchange(sh, im, R16Out<16>(), tid);
    r16<T, 256, DIR>(re, im, tw, tid);
    exchange(sh, re, R16Out<256>(), tid);
    exchange(sh, im, R16Out<256>(), tid);
    r4_last<T, DIR>(re, im, tw, tid);  // registers now hold X[tid + 1024 q]
}

// Z'_k from Z_k and its partner Z_{NC-k}.
template <typename T>
__device__ __forceinline__ void spectrum_one(T zr, T zi, T pr, T pi,
                                             typename Vec2T<T>::type w,
                                             typename Vec2T<T>::type c, T &outr, T &outi) {
    const T er = (zr + pr) * (T)0.5, ei = (zi - pi) * (T)0.5;    // E = (Z + conj Zp)/2
    const T orr = (zi + pi) * (T)0.5, oi = -(zr - pr) * (T)0.5;  // O = (Z - conj Zp)/2i
    const T wr = w.x, wi = w.y;                                  // W^k
    const T a1r = wr * orr - wi * oi, a1i = wr * oi + wi * orr;  // W^k O
    const T b1r = wr * er + wi * ei, b1i = wr * ei - wi * er;    // W^-k E
    const T sr = a1r - b1i, si = a1i + b1r;                      // W^k O + i W^-k E
    outr = c.x * zr + c.y * sr;
    outi = c.x * zi + c.y * si;
}

// Spectrum step on registers X[tid + 1024 q]: q < 8 is the lower half of the
// spectrum (k < NC/2), q >= 8 the upper half.  The upper half goes to LDS, both
// components.  The owner of each lower k reads its partner NC - k there and
// computes both outputs of the pair. It keeps Z'_k and writes Z'_{NC-k} over
// the partner's slot, which no other thread reads. Then every thread reads
// its upper half back.  Thread 0's q = 0 takes k = 0 and k = NC/2 (slot 0),
// each paired with itself.  Half the LDS traffic and three barriers, where
// moving both components to a pair layout and back takes eight.
template <typename T>
__device__ __forceinline__ void spectrum_step(T *__restrict__ sh, T (&re)[16], T (&im)[16],
                                              const typename Vec2T<T>::type *__restrict__ abf,
                                              const typename Vec2T<T>::type *__restrict__ twN,
                                              int tid) {
    constexpr int H = BNC / 2;
    T *shr = sh, *shi = sh + H;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        shr[tid + BTH * q] = re[8 + q];
        shi[tid + BTH * q] = im[8 + q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k1 = tid + BTH * q;
        const bool self = k1 == 0;
        const int k2 = self ? H : BNC - k1;
        const int u2 = k2 - H;  // LDS slot of k2
        const T z1r = re[q], z1i = im[q];
        const T z2r = shr[u2], z2i = shi[u2];
        T o1r, o1i, o2r, o2i;
        spectrum_one<T>(z1r, z1i, self ? z1r : z2r, self ? z1i : z2i, twN[k1], abf[k1], o1r, o1i);
        spectrum_one<T>(z2r, z2i, self ? z2r : z1r, self ? z2i : z1i, twN[k2], abf[k2], o2r, o2i);
        shr[u2] = o2r;
        shi[u2] = o2i;
        re[q] = o1r;
        im[q] = o1i;
        __builtin_amdgcn_sched_barrier(0);  // keep the table loads of one pair at a time
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        re[8 + q] = shr[tid + BTH * q];
        im[8 + q] = shi[tid + BTH * q];
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(BTH)
    k_noise_fft_big(const int64_t *__restrict__ blocks, const int64_t *__restrict__ istart,
                    const int32_t *__restrict__ fid,
                    const typename Vec2T<T>::type *__restrict__ ab,
                    const typename Vec2T<T>::type *__restrict__ tw,
                    const typename Vec2T<T>::type *__restrict__ twN, int lam, int V, int R,
                    const T *__restrict__ y, T *__restrict__ z) {
    __shared__ T sh[BLDS];
    const int tid = threadIdx.x;
    const int rr = blockIdx.y;
    const int64_t t0 = blocks[2 * blockIdx.x];
    const int64_t iv = blocks[2 * blockIdx.x + 1];
    const int64_t a = istart[iv], e = istart[iv + 1];
    const int64_t base = t0 - lam;
    T re[16], im[16];
    // forward pass 1 from global: z_m = y_{base+2m} + i y_{base+2m+1}, m = tid + 1024 r.
    // Block-uniform base pointer and bounds, 32-bit per-thread offsets.
    const T *yb = y + base * R + rr;
    const int lo = (int)(a - base), hi = (int)(e - base);  // valid offsets [lo, hi)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int u0 = 2 * (tid + BTH * r);
        re[r] = (u0 >= lo && u0 < hi) ? yb[u0 * R] : (T)0;
        im[r] = (u0 + 1 >= lo && u0 + 1 < hi) ? yb[(u0 + 1) * R] : (T)0;
    }
    dft16<T, -1>(re, im);
    passes_234<T, -1>(sh, re, im, tw, tid);

    // spectrum: Z'_k = A_k Z_k + B_k (W^k O_k + i W^-k E_k), with the partner
    // Z_{NC-k} exchanged through LDS.  Each phase below works from its own
    // opaque copy of the thread index, so the compiler recomputes the (cheap)
    // LDS addresses instead of keeping the forward half's addresses alive
    // across the whole transform.
    int tid_s = tid;
    asm volatile("" : "+v"(tid_s));
    spectrum_step<T>(sh, re, im, ab + (int64_t)fid[iv] * BNC, twN, tid_s);

    // inverse: pass 1 straight from the registers (inputs x[tid + 1024 r])
    int tid_i = tid;
    asm volatile("" : "+v"(tid_i));
    dft16<T, 1>(re, im);
    passes_234<T, 1>(sh, re, im, tw, tid_i);
    // registers hold z'_m, m = tid + 1024 q: outputs 2m and 2m + 1 of the block
    const int nvalid = (int)(e - t0 < V ? e - t0 : V);
    T *zb = z + t0 * R + rr;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int q0 = 2 * (tid_i + BTH * q) - lam;
        if (q0 >= 0 && q0 < nvalid) zb[q0 * R] = re[q];
        if (q0 + 1 >= 0 && q0 + 1 < nvalid) zb[(q0 + 1) * R] = im[q];
    }
}

}  // namespace

bool noise_fft_big_supported(int half_bw) { return half_bw >= 1 && half_bw <= BIG_MAX_LAMBDA; }
int noise_fft_big_nc() { return BNC; }

void noise_fft_big_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z) {
    Scope sc(ctx->prof, ctx->stream, "Ninv_fft");
    dim3 grid((unsigned)nz->n_fft_blocks, nrhs);
    if (nz->prec == MM_F32) {
        const float2 *tw = nz->fft_tw.as<float2>();
        k_noise_fft_big<float><<<grid, BTH, 0, ctx->stream>>>(
            nz->fft_blocks.as<int64_t>(), nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
            nz->fft_spec.as<float2>(), tw, tw + BNC, nz->half_bw, nz->fft_valid, nrhs,
            static_cast<const float *>(y), static_cast<float *>(z));
    } else {
        const double2 *tw = nz->fft_tw.as<double2>();
        k_noise_fft_big<double><<<grid, BTH, 0, ctx->stream>>>(
            nz->fft_blocks.as<int64_t>(), nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
            nz->fft_spec.as<double2>(), tw, tw + BNC, nz->half_bw, nz->fft_valid, nrhs,
            static_cast<const double *>(y), static_cast<double *>(z));
    }
    MM_HIP(hipGetLastError());
}

}  // namespace mm
