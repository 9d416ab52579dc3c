// N^-1 by FFT with register-resident overlap-save blocks of N = 2 NC real
// samples, packed as NC complex points (same packed-real scheme as
// noise_fft.hip), V = N - 2 lambda valid outputs.  Two sizes:
//   NC = 16,384 (N = 32,768): 1,024 threads, 128 KB of LDS -- one block per
//     CU; at lambda = 4,096 three quarters of every block are valid, and
//     bandwidths up to 12,288 fit;
//   NC = 8,192 (N = 16,384): 512 threads, 64 KB of LDS -- two blocks per CU,
//     so one block's memory phase overlaps the other's transforms; half of a
//     block is valid at lambda = 4,096, bandwidths up to 6,144 fit.
//
// Each thread holds 16 complex values in registers through the whole
// transform: radices 16 x 16 x 16 x RL with RL = NC / 4,096.  Between passes
// the values are exchanged through LDS one component at a time (real parts,
// then imaginary parts), so the exchange buffer is NC FP64 values
// (xor-swizzled) and the thread's other component stays in registers.  The
// first forward pass reads global memory, the radix-RL passes run in
// registers, the spectrum step reads each value's partner Z_{NC-k} through
// the same LDS buffer, and the last inverse pass writes global memory.  The
// block reads and writes global memory through raw buffer resources sized to
// its window and to its valid outputs, so the interval clipping and the
// overlap-save discard cost no per-element compares.
#include <cmath>

#include "fft_common.h"
#include "xcd.h"

namespace mm {
namespace {

using fft::dft4;
using fft::dft16;

// Transform geometry: NC complex points, TH = NC / 16 threads, last radix RL.
template <int NC_> struct Geo {
    static constexpr int NC = NC_;
    static constexpr int TH = NC_ / 16;
    static constexpr int RL = NC_ / 4096;
    static_assert(RL == 2 || RL == 4, "NC must be 8192 or 16384");
};
constexpr int BIG_MAX_LAMBDA = 12288;  // 32,768-sample blocks: V = N - 2 lambda >= 8,192
constexpr int MID_MAX_LAMBDA = 6144;   // 16,384-sample blocks: V >= 4,096

// Raw buffer accesses (resource word of the gfx9 family, stride 0): a load
// whose offset (VGPR part plus instruction offset) falls outside
// [0, num_records) bytes returns 0 and such a store is dropped.  A block's
// input resource covers its window clipped to the interval and its output
// resource the block's valid outputs, which gives the overlap-save block its
// zero padding and discards its edges with 32-bit offsets and no compares.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
// Two consecutive elements in one access (16 bytes FP64, 8 bytes FP32).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void buf_ld2(__amdgpu_buffer_rsrc_t r, int off, double &a, double &b) {
    const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void buf_ld2(__amdgpu_buffer_rsrc_t r, int off, float &a, float &b) {
    const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, int off, double a, double b) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, make_double2(a, b)), r, off,
                                           0, 0);
}
__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, int off, float a, float b) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, make_float2(a, b)), r, off, 0,
                                          0);
}

// LDS index of element i: its low four bits xor-ed with the next four, a
// bijection on [0, NC) that spreads the stride-16 accesses of the radix-16
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
// index tid + TH q.  The barrier that protects the LDS from being
// overwritten while other threads still read it sits before the stores
// (PRE), not after the loads, so that a wave goes on to its arithmetic as
// soon as its own loads are done; the first exchange of a block, with no
// earlier LDS use, has none.
template <typename G, typename T, bool PRE = true, typename F>
__device__ __forceinline__ void exchange(T *__restrict__ sh, T (&v)[16], const F &out, int tid) {
    if (PRE) __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) sh[padb(out(r, tid))] = v[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = sh[padb(tid + G::TH * q)];
}

// Radix-16 pass at sub-transform size NS on the thread's butterfly j = tid,
// whose inputs x[j + TH r] are the registers; twiddle then DFT, leaving the
// outputs for index (j/NS) NS 16 + j mod NS + r NS.
template <typename G, typename T, int NS, int DIR>
__device__ __forceinline__ void r16(T (&re)[16], T (&im)[16],
                                    const typename Vec2T<T>::type *__restrict__ tw, int tid) {
    if (NS > 1) {
        const int jm = tid % NS;
        const auto w = tw[jm * (G::NC / (NS * 16))];
        twiddle_seq<T, 16>(re, im, w.x, DIR < 0 ? w.y : -w.y);
    }
    dft16<T, DIR>(re, im);
}

template <int NS> struct R16Out {
    __device__ __forceinline__ int operator()(int r, int j) const {
        return (j / NS) * NS * 16 + (j % NS) + r * NS;
    }
};

// Last pass, radix RL at NS = 4096, entirely in registers: butterfly
// jj = tid + TH p (p < 16 / RL) takes x[jj + 4096 r] = register p + (16 / RL) r
// and writes it back in place.
template <typename G, typename T, int DIR>
__device__ __forceinline__ void r_last(T (&re)[16], T (&im)[16],
                                       const typename Vec2T<T>::type *__restrict__ tw, int tid) {
    constexpr int RL = G::RL, NP = 16 / RL;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int jj = tid + G::TH * p;
        T vr[RL], vi[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            vr[r] = re[p + NP * r];
            vi[r] = im[p + NP * r];
        }
        const auto w = tw[jj * (G::NC / (4096 * RL))];
        twiddle_seq<T, RL>(vr, vi, w.x, DIR < 0 ? w.y : -w.y);
        if constexpr (RL == 4) {
            dft4<T, DIR>(vr[0], vi[0], vr[1], vi[1], vr[2], vi[2], vr[3], vi[3]);
        } else {
            const T ar = vr[0] + vr[1], ai = vi[0] + vi[1];
            vr[1] = vr[0] - vr[1];
            vi[1] = vi[0] - vi[1];
            vr[0] = ar;
            vi[0] = ai;
        }
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            re[p + NP * r] = vr[r];
            im[p + NP * r] = vi[r];
        }
    }
}

// FIRST_PRE: whether the LDS may still be read by an earlier phase (the
// inverse transform, after the spectrum step) when the first exchange starts.
template <typename G, typename T, int DIR, bool FIRST_PRE>
__device__ __forceinline__ void passes_234(T *__restrict__ sh, T (&re)[16], T (&im)[16],
                                           const typename Vec2T<T>::type *__restrict__ tw,
                                           int tid) {
    // after pass 1 the registers hold outputs for index tid*16 + r
    exchange<G, T, FIRST_PRE>(sh, re, R16Out<1>(), tid);
    exchange<G>(sh, im, R16Out<1>(), tid);
    r16<G, T, 16, DIR>(re, im, tw, tid);
    exchange<G>(sh, re, R16Out<16>(), tid);
    exchange<G>(sh, im, R16Out<16>(), tid);
    r16<G, T, 256, DIR>(re, im, tw, tid);
    exchange<G>(sh, re, R16Out<256>(), tid);
    exchange<G>(sh, im, R16Out<256>(), tid);
    r_last<G, T, DIR>(re, im, tw, tid);  // registers now hold X[tid + TH q]
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

// Spectrum step on registers X[tid + TH q]: q < 8 is the lower half of the
// spectrum (k < NC/2), q >= 8 the upper half.  The upper half goes to LDS, both
// components.  The owner of each lower k reads its partner NC - k there and
// computes both outputs of the pair. It keeps Z'_k and writes Z'_{NC-k} over
// the partner's slot, which no other thread reads. Then every thread reads
// its upper half back.  Thread 0's q = 0 takes k = 0 and k = NC/2 (slot 0),
// each paired with itself.  Half the LDS traffic and two barriers, where
// moving both components to a pair layout and back takes eight.
template <typename G, typename T>
__device__ __forceinline__ void spectrum_step(T *__restrict__ sh, T (&re)[16], T (&im)[16],
                                              const typename Vec2T<T>::type *__restrict__ abf,
                                              const typename Vec2T<T>::type *__restrict__ twN,
                                              int tid) {
    constexpr int H = G::NC / 2;
    T *shr = sh, *shi = sh + H;
    // Element u of each half sits at padb(u).  Since H is a power of two
    // above the swizzle's bits, H + padb(u) = padb(H + u): a thread's stores
    // go to exactly the LDS words it loaded itself in the forward transform's
    // last exchange (indices tid + TH q, q < 16), so no barrier is needed
    // before them.
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        shr[padb(tid + G::TH * q)] = re[8 + q];
        shi[padb(tid + G::TH * q)] = im[8 + q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k1 = tid + G::TH * q;
        const bool self = k1 == 0;
        const int k2 = self ? H : G::NC - k1;
        const int u2 = k2 - H;  // LDS slot of k2
        const T z1r = re[q], z1i = im[q];
        const T z2r = shr[padb(u2)], z2i = shi[padb(u2)];
        T o1r, o1i, o2r, o2i;
        spectrum_one<T>(z1r, z1i, self ? z1r : z2r, self ? z1i : z2i, twN[k1], abf[k1], o1r, o1i);
        spectrum_one<T>(z2r, z2i, self ? z2r : z1r, self ? z2i : z1i, twN[k2], abf[k2], o2r, o2i);
        shr[padb(u2)] = o2r;
        shi[padb(u2)] = o2i;
        re[q] = o1r;
        im[q] = o1i;
        __builtin_amdgcn_sched_barrier(0);  // keep the table loads of one pair at a time
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        re[8 + q] = shr[padb(tid + G::TH * q)];
        im[8 + q] = shi[padb(tid + G::TH * q)];
    }
    // the inverse transform's first exchange waits for these loads
}

// RC = the column count when it is known at compile time (1), else 0 and the
// column count is R.
template <typename G, typename T, int RC>
__global__ void __launch_bounds__(G::TH) __attribute__((amdgpu_waves_per_eu(4)))
    k_noise_fft_reg(const int64_t *__restrict__ blocks, const int64_t *__restrict__ istart,
                    const int32_t *__restrict__ fid,
                    const typename Vec2T<T>::type *__restrict__ ab,
                    const typename Vec2T<T>::type *__restrict__ tw,
                    const typename Vec2T<T>::type *__restrict__ twN, int lam, int V, int R_,
                    int64_t n_blk, const T *__restrict__ y, T *__restrict__ z) {
    __shared__ T sh[G::NC];
    const int R = RC > 0 ? RC : R_;
    const int tid = threadIdx.x;
    // One flat grid of (block, column) pairs, padded to a multiple of 8 and
    // remapped so that each XCD takes a contiguous run of them.  Neighbouring
    // blocks of an interval then share their 2 lambda-sample halos, and the
    // blocks of one filter its spectrum table, in that XCD's L2 (one column:
    // 0.964 -> 0.945 ms at 2^27 samples, lambda 4,096); the R columns of a
    // block are neighbours too, and read and write the same interleaved
    // cache lines.  Padding blocks leave before any barrier.
    int64_t bx = blockIdx.x;
    int rr = 0;
    {
        const int64_t l = xcd_block(blockIdx.x, gridDim.x);
        if (l >= n_blk * R) return;
        bx = l / R;
        rr = (int)(l % R);
    }
    const int64_t t0 = blocks[2 * bx];
    const int64_t iv = blocks[2 * bx + 1];
    const int64_t a = istart[iv], e = istart[iv + 1];
    const int64_t base = t0 - lam;
    T re[16], im[16];
    // forward pass 1 from global: z_m = y_{base+2m} + i y_{base+2m+1}, m = tid + TH r.
    // The resource spans the window [base, base + 2 NC) clipped to the
    // interval [a, e): samples outside it read as 0.
    const int64_t w0 = base > a ? base : a;
    const int64_t w1 = base + 2 * G::NC < e ? base + 2 * G::NC : e;
    const auto ry = raw_rsrc(y + w0 * R, (w1 - w0) * R * (int64_t)sizeof(T));
    const int off0 = ((int)(base - w0) * R + rr) * (int)sizeof(T);
    // One column: each thread's pair (y_{2m}, y_{2m+1}) is one access when
    // the window's ends fall on even offsets from base, so that no pair
    // straddles them (block-uniform; false only for odd lambda or an odd
    // interval end).  Otherwise, and for several columns, every access moves
    // one element, wholly inside or outside the resource; the second
    // element's offset is hidden from the optimiser there so that the two
    // are never merged into one access across a resource end.
    if (RC == 1 && (((w0 - base) | (w1 - base)) & 1) == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            buf_ld2(ry, off0 + 2 * (tid + G::TH * r) * (int)sizeof(T), re[r], im[r]);
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int off = off0 + 2 * (tid + G::TH * r) * R * (int)sizeof(T);
            int off1 = off + R * (int)sizeof(T);
            asm volatile("" : "+v"(off1));
            re[r] = buf_ld<T>(ry, off);
            im[r] = buf_ld<T>(ry, off1);
        }
    }
    dft16<T, -1>(re, im);
    passes_234<G, T, -1, false>(sh, re, im, tw, tid);

    // spectrum: Z'_k = A_k Z_k + B_k (W^k O_k + i W^-k E_k), with the partner
    // Z_{NC-k} exchanged through LDS.  Each phase below works from its own
    // opaque copy of the thread index, so the compiler recomputes the (cheap)
    // LDS addresses instead of keeping the forward half's addresses alive
    // across the whole transform.
    int tid_s = tid;
    asm volatile("" : "+v"(tid_s));
    spectrum_step<G, T>(sh, re, im, ab + (int64_t)fid[iv] * G::NC, twN, tid_s);

    // inverse: pass 1 straight from the registers (inputs x[tid + TH r])
    int tid_i = tid;
    asm volatile("" : "+v"(tid_i));
    dft16<T, 1>(re, im);
    passes_234<G, T, 1, true>(sh, re, im, tw, tid_i);
    // registers hold z'_m, m = tid + TH q: outputs 2m and 2m + 1 of the block
    // output 2m - lam of the block is valid in [0, nvalid): the resource
    // spans exactly those outputs, the stores of the others are dropped
    const int64_t nvalid = e - t0 < V ? e - t0 : V;
    const auto rz = raw_rsrc(z + t0 * R, nvalid * R * (int64_t)sizeof(T));
    // pairs as for the loads: the valid range [0, nvalid) starts lam before
    // each pair's even offset 2m, so pairs are whole when lam and nvalid are even
    if (RC == 1 && ((lam | (int)nvalid) & 1) == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            buf_st2(rz, (2 * (tid_i + G::TH * q) - lam) * (int)sizeof(T), re[q], im[q]);
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int off = ((2 * (tid_i + G::TH * q) - lam) * R + rr) * (int)sizeof(T);
            int off1 = off + R * (int)sizeof(T);
            asm volatile("" : "+v"(off1));
            buf_st(rz, off, re[q]);
            buf_st(rz, off1, im[q]);
        }
    }
}

}  // namespace

bool noise_fft_big_supported(int half_bw) { return half_bw >= 1 && half_bw <= BIG_MAX_LAMBDA; }
bool noise_fft_mid_supported(int half_bw) { return half_bw >= 1 && half_bw <= MID_MAX_LAMBDA; }
int noise_fft_big_nc() { return Geo<16384>::NC; }
int noise_fft_mid_nc() { return Geo<8192>::NC; }

// Register-resident overlap-save apply with the block size the handle was
// prepared for (nz->fft_n = 32,768 or 16,384).
void noise_fft_reg_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z) {
    Scope sc(ctx->prof, ctx->stream, "Ninv_fft");
    // (block, column) pairs on a flat grid padded to a multiple of 8 (see
    // the kernel)
    const int64_t nb = nz->n_fft_blocks;
    const dim3 grid((unsigned)((nb * nrhs + 7) / 8 * 8));
    auto go = [&](auto GG) {
        using G = decltype(GG);
        if (nz->prec == MM_F32) {
            const float2 *tw = nz->fft_tw.as<float2>();
            auto k = nrhs == 1 ? k_noise_fft_reg<G, float, 1> : k_noise_fft_reg<G, float, 0>;
            k<<<grid, G::TH, 0, ctx->stream>>>(
                nz->fft_blocks.as<int64_t>(), nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
                nz->fft_spec.as<float2>(), tw, tw + G::NC, nz->half_bw, nz->fft_valid, nrhs, nb,
                static_cast<const float *>(y), static_cast<float *>(z));
        } else {
            const double2 *tw = nz->fft_tw.as<double2>();
            auto k = nrhs == 1 ? k_noise_fft_reg<G, double, 1> : k_noise_fft_reg<G, double, 0>;
            k<<<grid, G::TH, 0, ctx->stream>>>(
                nz->fft_blocks.as<int64_t>(), nz->istart.as<int64_t>(), nz->fid.as<int32_t>(),
                nz->fft_spec.as<double2>(), tw, tw + G::NC, nz->half_bw, nz->fft_valid, nrhs, nb,
                static_cast<const double *>(y), static_cast<double *>(z));
        }
    };
    if (nz->fft_n == 2 * Geo<16384>::NC) go(Geo<16384>());
    else go(Geo<8192>());
    MM_HIP(hipGetLastError());
}

}  // namespace mm
