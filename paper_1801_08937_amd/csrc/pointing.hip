// Pointing build: hit counts, observed-pixel selection, compact pixel ids, the
// pixel-sorted sample permutation with its CSR offsets, and the polarisation
// weights (cos 2psi, sin 2psi) of Eq. datamodel, all on the device.
//
// Integer work only apart from the weights, so every integer output is
// bit-exact and independent of scheduling: the histogram uses integer atomics
// (order does not change a sum of integers); the permutation comes from a
// stable LSD radix sort of (pixel, time).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "mm_internal.h"
#include "pol_weights.h"

namespace mm {
namespace {

constexpr int BS = 256;

__global__ void k_validate(const int32_t *__restrict__ pix, const double *__restrict__ psi,
                           int64_t n, int32_t npt, int *__restrict__ flags) {
    int bad_pix = 0, bad_psi = 0;
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        int32_t p = pix[t];
        bad_pix |= (p < -1 || p >= npt);
        if (psi) bad_psi |= !isfinite(psi[t]);
    }
    if (bad_pix) atomicOr(&flags[0], 1);
    if (bad_psi) atomicOr(&flags[1], 1);
}

__global__ void k_hist(const int32_t *__restrict__ pix, int64_t n, int32_t *__restrict__ hits) {
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        int32_t p = pix[t];
        if (p >= 0) atomicAdd(&hits[p], 1);
    }
}

__global__ void k_obs_flag(const int32_t *__restrict__ hits, int32_t npt, int32_t min_hits,
                           int32_t *__restrict__ flag) {
    int32_t p = blockIdx.x * BS + threadIdx.x;
    if (p < npt) flag[p] = hits[p] >= min_hits ? 1 : 0;
}

// cidx[p] = rank among observed pixels (exclusive scan of flags), -1 if not
// observed; obs_pix[rank] = p; obs_hits[rank] = hits[p]; obs_hits[n_obs] = 0.
__global__ void k_compact(const int32_t *__restrict__ hits, const int32_t *__restrict__ flag,
                          const int32_t *__restrict__ scan, int32_t npt,
                          int32_t *__restrict__ cidx, int32_t *__restrict__ obs_pix,
                          int32_t *__restrict__ obs_hits) {
    int32_t p = blockIdx.x * BS + threadIdx.x;
    if (p >= npt) return;
    if (flag[p]) {
        int32_t c = scan[p];
        cidx[p] = c;
        obs_pix[c] = p;
        obs_hits[c] = hits[p];
    } else {
        cidx[p] = -1;
    }
    if (p == npt - 1) obs_hits[scan[p] + flag[p]] = 0;
}

__global__ void k_sample_j(const int32_t *__restrict__ pix, const int32_t *__restrict__ cidx,
                           int64_t n, uint32_t flagged_key, int32_t *__restrict__ j,
                           uint32_t *__restrict__ keys, int32_t *__restrict__ vals) {
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        int32_t p = pix[t];
        int32_t c = p >= 0 ? cidx[p] : -1;
        j[t] = c;
        keys[t] = c >= 0 ? (uint32_t)c : flagged_key;
        vals[t] = (int32_t)t;
    }
}

template <typename T2>
__global__ void k_weights(const double *__restrict__ psi, int64_t n, T2 *__restrict__ w) {
    using T = decltype(T2::x);
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        double s, c;
        pol_weights(psi[t], c, s);
        T2 v;
        v.x = (T)c;
        v.y = (T)s;
        w[t] = v;
    }
}

template <typename T2>
__global__ void k_gather_w(const int32_t *__restrict__ perm, const T2 *__restrict__ w, int64_t n,
                           T2 *__restrict__ ws) {
    for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        ws[i] = w[perm[i]];
}

// order[s] = compact pixel visited s-th when P^T walks the observed pixels in
// square tiles of a row-major grid of the given width: key = (tile row, tile
// column, row in tile, column in tile) of the global id.
__global__ void k_tile_keys(const int32_t *__restrict__ obs_pix, int32_t n_obs, int32_t width,
                            int32_t tile, uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    const int32_t c = blockIdx.x * BS + threadIdx.x;
    if (c >= n_obs) return;
    const int64_t g = obs_pix[c];
    const int64_t y = g / width, x = g % width;
    const int64_t tiles_x = (width + tile - 1) / tile;
    const uint64_t k = ((uint64_t)((y / tile) * tiles_x + x / tile) << 24) |
                       (uint64_t)((y % tile) * tile + (x % tile));
    keys[c] = k;
    vals[c] = c;
}

// slot[order[r]] = r
__global__ void k_rank(const int32_t *__restrict__ order, int32_t n, int32_t *__restrict__ slot) {
    const int32_t r = blockIdx.x * BS + threadIdx.x;
    if (r < n) slot[order[r]] = r;
}
// Scan direction of each chunk of DIR_CHUNK consecutive samples: the
// displacement over DIR_STEP samples, where both ends are observed, at most
// DIR_MAXD pixels and not zero, votes for one of DIR_BINS angle bins over
// [0, 180) degrees; the chunk takes the bin with most votes (the lowest on a
// tie), or -1 without any vote.  Integer counts only, so the result does not
// depend on scheduling.
constexpr int DIR_CHUNK = 4096;
constexpr int DIR_STEP = 8;
constexpr int DIR_MAXD = 12;
constexpr int DIR_BINS = 12;
__global__ void __launch_bounds__(BS) k_chunk_dir(const int32_t *__restrict__ j,
                                                  const int32_t *__restrict__ obs_pix, int64_t n,
                                                  int32_t width, int32_t *__restrict__ bin) {
    __shared__ int cnt[DIR_BINS];
    if (threadIdx.x < DIR_BINS) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * DIR_CHUNK;
    const int64_t c1 = min(c0 + DIR_CHUNK, n) - DIR_STEP;
    for (int64_t t = c0 + threadIdx.x; t < c1; t += BS) {
        const int32_t a = j[t], b = j[t + DIR_STEP];
        if (a < 0 || b < 0) continue;
        const int32_t ga = obs_pix[a], gb = obs_pix[b];
        const int dx = gb % width - ga % width, dy = gb / width - ga / width;
        if ((dx == 0 && dy == 0) || abs(dx) > DIR_MAXD || abs(dy) > DIR_MAXD) continue;
        float ang = atan2f((float)dy, (float)dx) * (180.0f / 3.14159265f);
        if (ang < 0) ang += 180.0f;
        int k = (int)(ang * (DIR_BINS / 180.0f));
        k = k < 0 ? 0 : (k >= DIR_BINS ? DIR_BINS - 1 : k);
        atomicAdd(&cnt[k], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best = -1, bc = 0;
        for (int k = 0; k < DIR_BINS; ++k)
            if (cnt[k] > bc) {
                bc = cnt[k];
                best = k;
            }
        bin[blockIdx.x] = best;
    }
}

// First sample of each copy's samples that hits each pixel:
// first[g n_obs + c] = min t over samples t of copy g with pixel c.
__global__ void k_first_touch(const int32_t *__restrict__ j, const int32_t *__restrict__ grp,
                              int64_t n, int32_t n_obs,
                              unsigned long long *__restrict__ first) {
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        const int32_t c = j[t];
        if (c < 0) continue;
        const int64_t g = grp[t / DIR_CHUNK];
        atomicMin(&first[g * n_obs + c], (unsigned long long)t);
    }
}

// Sort keys: copy in the top byte, then the first touch (unhit pixels last,
// in compact id order through the stable sort); value = g n_obs + c.
__global__ void k_touch_keys(const unsigned long long *__restrict__ first, int64_t total,
                             int32_t n_obs, uint64_t *__restrict__ keys,
                             int32_t *__restrict__ vals) {
    for (int64_t e = blockIdx.x * (int64_t)BS + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * BS) {
        const uint64_t g = (uint64_t)(e / n_obs);
        const uint64_t f = first[e];
        keys[e] = (g << 56) | (f < (1ull << 56) ? f : (1ull << 56) - 1);
        vals[e] = (int32_t)e;
    }
}

// p_j[t] = slot of sample t's pixel in its chunk's copy (-1 flagged).
__global__ void k_slot_of_sample_g(const int32_t *__restrict__ j, const int32_t *__restrict__ grp,
                                   const int32_t *__restrict__ slot, int64_t n, int32_t n_obs,
                                   int32_t *__restrict__ pj) {
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        const int32_t c = j[t];
        pj[t] = c >= 0 ? slot[(int64_t)grp[t / DIR_CHUNK] * n_obs + c] : -1;
    }
}

// Sliced P^T layout.  Lane (g, l) finds, by binary search in its pixel's
// time-sorted list perm[off[c], off[c+1]), where each time segment
// [n s / S, n (s+1) / S) starts; cnt / start are stored per (s G + g, l).
// Sliced P^T per scan direction.  Sort keys of the pixel-sorted samples by
// their chunk's direction (a stable sort keeps pixel, then time, order inside
// each direction), the sample counts of every virtual pixel d n_obs + c, and
// the lane pixels: copy d's first-touch order of the pixels, a block of G
// slices per direction.
__global__ void k_perm_dir_keys(const int32_t *__restrict__ perm, int64_t n_valid,
                                const int32_t *__restrict__ grp, uint32_t *__restrict__ keys,
                                int32_t *__restrict__ vals) {
    for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n_valid;
         i += (int64_t)gridDim.x * BS) {
        keys[i] = (uint32_t)grp[perm[i] / DIR_CHUNK];
        vals[i] = (int32_t)i;
    }
}
__global__ void k_dir_counts(const int32_t *__restrict__ j, const int32_t *__restrict__ grp,
                             int64_t n, int32_t n_obs, int32_t *__restrict__ cnt) {
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        const int32_t c = j[t];
        if (c >= 0) atomicAdd(&cnt[(int64_t)grp[t / DIR_CHUNK] * n_obs + c], 1);
    }
}
template <typename V>
__global__ void k_perm_gather(const int32_t *__restrict__ idx, const int32_t *__restrict__ perm,
                              const V *__restrict__ w, int64_t n_valid,
                              int32_t *__restrict__ perm2, V *__restrict__ w2) {
    for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n_valid;
         i += (int64_t)gridDim.x * BS) {
        const int32_t k = idx[i];
        perm2[i] = perm[k];
        if (w) w2[i] = w[k];
    }
}
__global__ void k_sl_pix_dir(const int32_t *__restrict__ slot, int64_t total, int32_t n_obs,
                             int32_t G, int32_t *__restrict__ sl_pix) {
    for (int64_t v = blockIdx.x * (int64_t)BS + threadIdx.x; v < total;
         v += (int64_t)gridDim.x * BS) {
        const int64_t d = v / n_obs;
        const int64_t r = slot[v] - d * n_obs;  // rank in copy d
        sl_pix[d * G * 64 + r] = (int32_t)v;
    }
}

__global__ void k_sl_bounds(const int32_t *__restrict__ sl_pix, int32_t G, int32_t S,
                            int64_t n_samp, const int32_t *__restrict__ off,
                            const int32_t *__restrict__ perm, int32_t *__restrict__ cnt,
                            int32_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= (int64_t)G * 64) return;
    const int64_t g = i >> 6, l = i & 63;
    const int32_t c = sl_pix[i];
    int32_t prev = c >= 0 ? off[c] : 0;
    const int32_t end = c >= 0 ? off[c + 1] : 0;
    for (int32_t sg = 0; sg < S; ++sg) {
        int32_t hi = end;
        if (sg + 1 < S) {
            const int64_t T = n_samp * (sg + 1) / S;
            int32_t lo = prev;
            hi = end;
            while (lo < hi) {  // first entry with perm >= T
                const int32_t mid = lo + ((hi - lo) >> 1);
                if (perm[mid] < T)
                    lo = mid + 1;
                else
                    hi = mid;
            }
        }
        const int64_t o = ((int64_t)sg * G + g) * 64 + l;
        cnt[o] = hi - prev;
        start[o] = prev;
        prev = hi;
    }
}

// sizes[w] = 64 x (largest lane count of wave w); sizes[n_waves] = 0.
__global__ void k_sl_width(const int32_t *__restrict__ cnt, int64_t n_waves,
                           int64_t *__restrict__ sizes) {
    const int64_t w = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w > n_waves) return;
    if (w == n_waves) {
        if (lane == 0) sizes[w] = 0;
        return;
    }
    int32_t m = cnt[w * 64 + lane];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d));
    if (lane == 0) sizes[w] = 64 * (int64_t)m;
}

// Entries of wave w: lane l's k-th sample of its pixel in the segment (or
// padding).  V is the per-entry weight record: the stored weights (FP32
// form) or the angle psi gathered from time order (FP64 form, weights formed
// on the fly).
template <typename V>
__device__ __forceinline__ V sl_value(const V *__restrict__ src, int64_t i, int32_t t) {
    return src[i];
}
template <>
__device__ __forceinline__ double sl_value<double>(const double *__restrict__ psi, int64_t,
                                                   int32_t t) {
    return psi[t];
}
__device__ __forceinline__ void sl_zero(float2 &v) { v = make_float2(0.f, 0.f); }
__device__ __forceinline__ void sl_zero(double &v) { v = 0.0; }

template <typename V>
__global__ void k_sl_fill(const int64_t *__restrict__ base, const int32_t *__restrict__ cnt,
                          const int32_t *__restrict__ start, const int32_t *__restrict__ perm,
                          const V *__restrict__ src, int64_t n_waves,
                          int32_t *__restrict__ sl_perm, V *__restrict__ sl_w) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * BS) >> 6;
    for (int64_t w = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6; w < n_waves; w += nw) {
        const int64_t b0 = base[w];
        const int64_t W = (base[w + 1] - b0) >> 6;
        const int32_t c = cnt[w * 64 + lane];
        const int32_t st = start[w * 64 + lane];
        for (int64_t k = 0; k < W; ++k) {
            const int64_t idx = b0 + 64 * k + lane;
            if (k < c) {
                const int32_t t = perm[st + k];
                sl_perm[idx] = t;
                sl_w[idx] = sl_value<V>(src, st + k, t);
            } else {
                V zero;
                sl_zero(zero);
                sl_perm[idx] = -1;
                sl_w[idx] = zero;
            }
        }
    }
}

int grid_for(int64_t n, int max_blocks = 8192) {
    int64_t g = (n + BS - 1) / BS;
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

// Map copies of the single-column IQU P (width > 0), or none.  The lanes of
// a wave gather the map at consecutive samples, i.e. along the scan, so the
// gather touches few cache lines when pixels met one after the other along
// the scan sit next to each other in memory.  One order cannot do that for
// several scan directions, so the map is kept in up to MAX_COPIES copies,
// one per scan direction found (chunks of samples voting by their
// displacement), each ordered by the first sample of its chunks that hits
// each pixel.  The values gathered, hence P's output, do not depend on it.
constexpr int MAX_COPIES = 4;

void pointing_p_slots_device(mm_ctx *ctx, mm_pointing *p, int32_t width) {
    hipStream_t s = ctx->stream;
    p->p_slot.release();
    p->p_j.release();
    p->p_chunk_grp.release();
    p->p_copies = 0;
    const int32_t n_obs = p->n_obs;
    if (width <= 0 || n_obs == 0 || p->nc != 3) return;
    const int64_t n = p->n_samp;
    const int64_t n_chunks = (n + DIR_CHUNK - 1) / DIR_CHUNK;
    DBuf dbin;
    dbin.alloc(sizeof(int32_t) * n_chunks);
    k_chunk_dir<<<(unsigned)n_chunks, BS, 0, s>>>(p->j.as<int32_t>(), p->obs_pix.as<int32_t>(), n,
                                                  width, dbin.as<int32_t>());
    MM_HIP(hipGetLastError());
    std::vector<int32_t> bin(n_chunks);
    MM_HIP(hipMemcpyAsync(bin.data(), dbin.ptr, sizeof(int32_t) * n_chunks,
                          hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    // directions holding at least 1/16 of the directed chunks, most first; a
    // bin next to a kept one is not kept (a direction on a bin boundary
    // splits its chunks between two bins)
    int64_t cnt[DIR_BINS] = {};
    int64_t directed = 0;
    for (int32_t b : bin)
        if (b >= 0) {
            ++cnt[b];
            ++directed;
        }
    std::vector<int> kept;
    {
        std::vector<int> byc(DIR_BINS);
        for (int k = 0; k < DIR_BINS; ++k) byc[k] = k;
        std::stable_sort(byc.begin(), byc.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
        for (int k : byc) {
            if (cnt[k] == 0 || cnt[k] * 16 < directed || (int)kept.size() == MAX_COPIES) continue;
            bool near = false;
            for (int q : kept) {
                const int d = std::abs(k - q);
                near |= std::min(d, DIR_BINS - d) <= 1;
            }
            if (!near) kept.push_back(k);
        }
    }
    int G = kept.empty() ? 1 : (int)kept.size();
    if ((int64_t)G * n_obs >= (int64_t)1 << 31) G = 1;
    // each chunk to the copy of the nearest kept direction (angles mod 180),
    // undirected chunks to the most common one
    std::vector<int32_t> grp(n_chunks, 0);
    if (G > 1)
        for (int64_t c = 0; c < n_chunks; ++c) {
            if (bin[c] < 0) continue;
            int bg = 0, bd = DIR_BINS;
            for (int g = 0; g < G; ++g) {
                int d = std::abs(bin[c] - kept[g]);
                d = std::min(d, DIR_BINS - d);
                if (d < bd) {
                    bd = d;
                    bg = g;
                }
            }
            grp[c] = bg;
        }
    DBuf first, keys, vals, ko, order, tmp;
    DBuf &dgrp = p->p_chunk_grp;
    dgrp.alloc(sizeof(int32_t) * n_chunks);
    MM_HIP(hipMemcpyAsync(dgrp.ptr, grp.data(), sizeof(int32_t) * n_chunks,
                          hipMemcpyHostToDevice, s));
    const int64_t total = (int64_t)G * n_obs;
    first.alloc(sizeof(unsigned long long) * total);
    MM_HIP(hipMemsetAsync(first.ptr, 0xff, sizeof(unsigned long long) * total, s));
    k_first_touch<<<grid_for(n), BS, 0, s>>>(p->j.as<int32_t>(), dgrp.as<int32_t>(), n, n_obs,
                                             first.as<unsigned long long>());
    keys.alloc(sizeof(uint64_t) * total);
    vals.alloc(sizeof(int32_t) * total);
    ko.alloc(sizeof(uint64_t) * total);
    order.alloc(sizeof(int32_t) * total);
    k_touch_keys<<<grid_for(total), BS, 0, s>>>(first.as<unsigned long long>(), total, n_obs,
                                                keys.as<uint64_t>(), vals.as<int32_t>());
    size_t tb = 0;
    MM_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys.as<uint64_t>(), ko.as<uint64_t>(),
                                     vals.as<int32_t>(), order.as<int32_t>(), (size_t)total, 0u,
                                     64u, s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tb, keys.as<uint64_t>(), ko.as<uint64_t>(),
                                     vals.as<int32_t>(), order.as<int32_t>(), (size_t)total, 0u,
                                     64u, s));
    // copy g's slots are [g n_obs, (g + 1) n_obs): the key's top byte is g
    p->p_slot.alloc(sizeof(int32_t) * total);
    k_rank<<<(unsigned)((total + BS - 1) / BS), BS, 0, s>>>(order.as<int32_t>(), (int32_t)total,
                                                           p->p_slot.as<int32_t>());
    p->p_j.alloc(sizeof(int32_t) * n);
    k_slot_of_sample_g<<<grid_for(n), BS, 0, s>>>(p->j.as<int32_t>(), dgrp.as<int32_t>(),
                                                  p->p_slot.as<int32_t>(), n, n_obs,
                                                  p->p_j.as<int32_t>());
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(s));
    p->p_copies = G;
}

void pointing_set_grid_device(mm_ctx *ctx, mm_pointing *p, int32_t width, int32_t tile) {
    hipStream_t s = ctx->stream;
    const int32_t n_obs = p->n_obs;
    if (n_obs == 0) return;
    DBuf keys, vals, ko, vo, tmp;
    keys.alloc(sizeof(uint64_t) * n_obs);
    vals.alloc(sizeof(int32_t) * n_obs);
    ko.alloc(sizeof(uint64_t) * n_obs);
    p->seg_order.alloc(sizeof(int32_t) * n_obs);
    k_tile_keys<<<(n_obs + BS - 1) / BS, BS, 0, s>>>(p->obs_pix.as<int32_t>(), n_obs, width, tile,
                                                     keys.as<uint64_t>(), vals.as<int32_t>());
    size_t tb = 0;
    MM_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys.as<uint64_t>(), ko.as<uint64_t>(),
                                     vals.as<int32_t>(), p->seg_order.as<int32_t>(),
                                     (size_t)n_obs, 0u, 64u, s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tb, keys.as<uint64_t>(), ko.as<uint64_t>(),
                                     vals.as<int32_t>(), p->seg_order.as<int32_t>(),
                                     (size_t)n_obs, 0u, 64u, s));
    MM_HIP(hipStreamSynchronize(s));
}

// Time segments for the sliced P^T: enough (segment, slice) waves to fill
// the device (8,192 = 32 per CU on 256 CUs), and at least one segment per 2^22
// samples of time, so that the stretch of the TOD the resident waves gather from at
// any moment stays small enough for the L2 (at 1.34e8 samples: 32 segments,
// measured best among 8..128); at most 64, and at least 32 entries per lane,
// segment and scan direction on average.  A function of the problem size only, so the
// summation order (and the bits of the result) does not depend on the device.
static int32_t slice_segments(int64_t n_samp, int64_t n_valid, int32_t n_obs, int32_t G,
                              int32_t D) {
    int64_t S = 8192 / G;
    if (S < (n_samp >> 22)) S = n_samp >> 22;
    if (S > 64) S = 64;
    const int64_t cap = n_obs > 0 ? n_valid / n_obs / 32 / D : 0;
    if (S > cap) S = cap;
    return (int32_t)(S < 1 ? 1 : S);
}

void pointing_slices_device(mm_ctx *ctx, mm_pointing *p, int32_t width) {
    hipStream_t s = ctx->stream;
    p->sl_G = p->sl_S = 0;
    p->sl_D = 1;
    p->sl_pix.release();
    p->sl_base.release();
    p->sl_perm.release();
    p->sl_w.release();
    const int32_t n_obs = p->n_obs;
    // IQU only: the I and QU pointings reduce with the one-wave-per-pixel form
    if (n_obs == 0 || p->n_valid == 0 || p->nc != 3) return;
    const int32_t G0 = (n_obs + 63) / 64;
    // below ~2,048 waves the one-wave-per-pixel kernel is the faster one
    if ((int64_t)G0 * slice_segments(p->n_samp, p->n_valid, n_obs, G0, 1) < 2048) return;
    // per scan direction when the map copies of P are there
    const bool dirs = width > 0 && p->p_copies > 0 && p->p_chunk_grp.ptr;
    const int32_t D = dirs ? p->p_copies : 1;
    const int32_t S = slice_segments(p->n_samp, p->n_valid, n_obs, G0, D);
    const int32_t G = G0 * D;
    const int64_t nv = p->n_valid;
    const bool f32 = p->prec == MM_F32;
    // the pixel-sorted samples and their CSR offsets, over virtual pixels
    // d n_obs + c when cut by direction
    const int32_t *perm_u = p->perm.as<int32_t>();
    const int32_t *off_u = p->off.as<int32_t>();
    const void *ws_u = f32 ? p->ws.ptr : nullptr;
    DBuf perm2, off2, ws2;
    if (dirs && D > 1) {
        DBuf keys, vals, ko, idx, cnt2, tmp;
        keys.alloc(sizeof(uint32_t) * nv);
        vals.alloc(sizeof(int32_t) * nv);
        ko.alloc(sizeof(uint32_t) * nv);
        idx.alloc(sizeof(int32_t) * nv);
        k_perm_dir_keys<<<grid_for(nv), BS, 0, s>>>(perm_u, nv, p->p_chunk_grp.as<int32_t>(),
                                                   keys.as<uint32_t>(), vals.as<int32_t>());
        size_t tb = 0;
        MM_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys.as<uint32_t>(), ko.as<uint32_t>(),
                                         vals.as<int32_t>(), idx.as<int32_t>(), (size_t)nv, 0u,
                                         8u, s));
        tmp.alloc(tb + 16);
        MM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tb, keys.as<uint32_t>(), ko.as<uint32_t>(),
                                         vals.as<int32_t>(), idx.as<int32_t>(), (size_t)nv, 0u,
                                         8u, s));
        perm2.alloc(sizeof(int32_t) * nv);
        if (f32) {
            ws2.alloc(sizeof(float2) * nv);
            k_perm_gather<float2><<<grid_for(nv), BS, 0, s>>>(
                idx.as<int32_t>(), perm_u, p->ws.as<float2>(), nv, perm2.as<int32_t>(),
                ws2.as<float2>());
        } else {
            k_perm_gather<float2><<<grid_for(nv), BS, 0, s>>>(
                idx.as<int32_t>(), perm_u, nullptr, nv, perm2.as<int32_t>(), nullptr);
        }
        const int64_t nvp = (int64_t)D * n_obs;
        cnt2.alloc(sizeof(int32_t) * (nvp + 1));
        MM_HIP(hipMemsetAsync(cnt2.ptr, 0, sizeof(int32_t) * (nvp + 1), s));
        k_dir_counts<<<grid_for(p->n_samp), BS, 0, s>>>(p->j.as<int32_t>(),
                                                        p->p_chunk_grp.as<int32_t>(), p->n_samp,
                                                        n_obs, cnt2.as<int32_t>());
        off2.alloc(sizeof(int32_t) * (nvp + 1));
        size_t tb2 = 0;
        MM_HIP(rocprim::exclusive_scan(nullptr, tb2, cnt2.as<int32_t>(), off2.as<int32_t>(),
                                       (int32_t)0, (size_t)(nvp + 1), rocprim::plus<int32_t>(),
                                       s));
        DBuf tmp2;
        tmp2.alloc(tb2 + 16);
        MM_HIP(rocprim::exclusive_scan(tmp2.ptr, tb2, cnt2.as<int32_t>(), off2.as<int32_t>(),
                                       (int32_t)0, (size_t)(nvp + 1), rocprim::plus<int32_t>(),
                                       s));
        MM_HIP(hipStreamSynchronize(s));
        perm_u = perm2.as<int32_t>();
        off_u = off2.as<int32_t>();
        if (f32) ws_u = ws2.ptr;
    }

    p->sl_pix.alloc(sizeof(int32_t) * (size_t)G * 64);
    MM_HIP(hipMemsetAsync(p->sl_pix.ptr, 0xff, sizeof(int32_t) * (size_t)G * 64, s));
    if (dirs) {
        const int64_t nvp = (int64_t)D * n_obs;
        k_sl_pix_dir<<<grid_for(nvp), BS, 0, s>>>(p->p_slot.as<int32_t>(), nvp, n_obs, G0,
                                                  p->sl_pix.as<int32_t>());
        MM_HIP(hipStreamSynchronize(s));
    } else if (width > 0) {
        DBuf keys, vals, ko;
        keys.alloc(sizeof(uint64_t) * n_obs);
        vals.alloc(sizeof(int32_t) * n_obs);
        ko.alloc(sizeof(uint64_t) * n_obs);
        k_tile_keys<<<(n_obs + BS - 1) / BS, BS, 0, s>>>(p->obs_pix.as<int32_t>(), n_obs, width, 8,
                                                         keys.as<uint64_t>(), vals.as<int32_t>());
        size_t tb = 0;
        MM_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys.as<uint64_t>(), ko.as<uint64_t>(),
                                         vals.as<int32_t>(), p->sl_pix.as<int32_t>(),
                                         (size_t)n_obs, 0u, 64u, s));
        DBuf tmp;
        tmp.alloc(tb + 16);
        MM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tb, keys.as<uint64_t>(), ko.as<uint64_t>(),
                                         vals.as<int32_t>(), p->sl_pix.as<int32_t>(),
                                         (size_t)n_obs, 0u, 64u, s));
        MM_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<int32_t> id(n_obs);
        for (int32_t c = 0; c < n_obs; ++c) id[c] = c;
        MM_HIP(hipMemcpyAsync(p->sl_pix.ptr, id.data(), sizeof(int32_t) * n_obs,
                              hipMemcpyHostToDevice, s));
        MM_HIP(hipStreamSynchronize(s));
    }

    const int64_t n_waves = (int64_t)G * S;
    DBuf cnt, start, sizes, tmp;
    cnt.alloc(sizeof(int32_t) * n_waves * 64);
    start.alloc(sizeof(int32_t) * n_waves * 64);
    sizes.alloc(sizeof(int64_t) * (n_waves + 1));
    p->sl_base.alloc(sizeof(int64_t) * (n_waves + 1));
    k_sl_bounds<<<(unsigned)((G * 64 + BS - 1) / BS), BS, 0, s>>>(
        p->sl_pix.as<int32_t>(), G, S, p->n_samp, off_u, perm_u, cnt.as<int32_t>(),
        start.as<int32_t>());
    k_sl_width<<<(unsigned)((n_waves + 1) * 64 / BS + 1), BS, 0, s>>>(cnt.as<int32_t>(), n_waves,
                                                                      sizes.as<int64_t>());
    size_t tb = 0;
    MM_HIP(rocprim::exclusive_scan(nullptr, tb, sizes.as<int64_t>(), p->sl_base.as<int64_t>(),
                                   (int64_t)0, (size_t)(n_waves + 1), rocprim::plus<int64_t>(),
                                   s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::exclusive_scan(tmp.ptr, tb, sizes.as<int64_t>(), p->sl_base.as<int64_t>(),
                                   (int64_t)0, (size_t)(n_waves + 1), rocprim::plus<int64_t>(),
                                   s));
    int64_t total = 0;
    MM_HIP(hipMemcpyAsync(&total, p->sl_base.as<int64_t>() + n_waves, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    p->sl_perm.alloc(sizeof(int32_t) * (size_t)total);
    p->sl_w.alloc((f32 ? sizeof(float2) : sizeof(double)) * (size_t)total);
    const unsigned fb = (unsigned)std::min<int64_t>((n_waves * 64 + BS - 1) / BS, 16384);
    if (f32)
        k_sl_fill<float2><<<fb, BS, 0, s>>>(p->sl_base.as<int64_t>(), cnt.as<int32_t>(),
                                            start.as<int32_t>(), perm_u,
                                            static_cast<const float2 *>(ws_u), n_waves,
                                            p->sl_perm.as<int32_t>(), p->sl_w.as<float2>());
    else
        k_sl_fill<double><<<fb, BS, 0, s>>>(p->sl_base.as<int64_t>(), cnt.as<int32_t>(),
                                            start.as<int32_t>(), perm_u, p->psi.as<double>(),
                                            n_waves, p->sl_perm.as<int32_t>(),
                                            p->sl_w.as<double>());
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(s));
    p->sl_G = G;
    p->sl_S = S;
    p->sl_D = D;
}

void pointing_build_device(mm_ctx *ctx, mm_pointing *p, const int32_t *pix, const double *psi,
                           int32_t min_hits) {
    hipStream_t s = ctx->stream;
    const int64_t n = p->n_samp;
    const int32_t npt = p->n_pix_total;

    DBuf flags;
    flags.alloc(2 * sizeof(int));
    MM_HIP(hipMemsetAsync(flags.ptr, 0, 2 * sizeof(int), s));
    k_validate<<<grid_for(n), BS, 0, s>>>(pix, psi, n, npt, flags.as<int>());
    int hf[2];
    MM_HIP(hipMemcpyAsync(hf, flags.ptr, sizeof(hf), hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    MM_CHECK(!hf[0], MM_E_INVALID, "pointing: pixel index outside [-1, n_pix_total)");
    MM_CHECK(!hf[1], MM_E_NONFINITE, "pointing: non-finite angle psi");

    p->hits.alloc(sizeof(int32_t) * npt);
    MM_HIP(hipMemsetAsync(p->hits.ptr, 0, sizeof(int32_t) * npt, s));
    k_hist<<<grid_for(n), BS, 0, s>>>(pix, n, p->hits.as<int32_t>());

    DBuf flag, scan, cidx, obs_hits_tmp, tmp;
    flag.alloc(sizeof(int32_t) * npt);
    scan.alloc(sizeof(int32_t) * npt);
    k_obs_flag<<<(npt + BS - 1) / BS, BS, 0, s>>>(p->hits.as<int32_t>(), npt, min_hits,
                                                   flag.as<int32_t>());
    size_t tb = 0;
    MM_HIP(rocprim::exclusive_scan(nullptr, tb, flag.as<int32_t>(), scan.as<int32_t>(), 0,
                                   (size_t)npt, rocprim::plus<int32_t>(), s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::exclusive_scan(tmp.ptr, tb, flag.as<int32_t>(), scan.as<int32_t>(), 0,
                                   (size_t)npt, rocprim::plus<int32_t>(), s));
    int32_t last[2];
    MM_HIP(hipMemcpyAsync(&last[0], scan.as<int32_t>() + npt - 1, 4, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(&last[1], flag.as<int32_t>() + npt - 1, 4, hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    const int32_t n_obs = last[0] + last[1];
    p->n_obs = n_obs;

    cidx.alloc(sizeof(int32_t) * npt);
    p->obs_pix.alloc(sizeof(int32_t) * (n_obs > 0 ? n_obs : 1));
    obs_hits_tmp.alloc(sizeof(int32_t) * (n_obs + 1));
    k_compact<<<(npt + BS - 1) / BS, BS, 0, s>>>(p->hits.as<int32_t>(), flag.as<int32_t>(),
                                                  scan.as<int32_t>(), npt, cidx.as<int32_t>(),
                                                  p->obs_pix.as<int32_t>(),
                                                  obs_hits_tmp.as<int32_t>());
    p->off.alloc(sizeof(int32_t) * (n_obs + 1));
    tb = 0;
    MM_HIP(rocprim::exclusive_scan(nullptr, tb, obs_hits_tmp.as<int32_t>(), p->off.as<int32_t>(),
                                   0, (size_t)(n_obs + 1), rocprim::plus<int32_t>(), s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::exclusive_scan(tmp.ptr, tb, obs_hits_tmp.as<int32_t>(), p->off.as<int32_t>(),
                                   0, (size_t)(n_obs + 1), rocprim::plus<int32_t>(), s));
    int32_t nv;
    MM_HIP(hipMemcpyAsync(&nv, p->off.as<int32_t>() + n_obs, 4, hipMemcpyDeviceToHost, s));

    // compact pixel per sample and the sort keys (flagged samples sort last)
    p->j.alloc(sizeof(int32_t) * n);
    DBuf keys, vals, keys_out, vals_out;
    keys.alloc(sizeof(uint32_t) * n);
    vals.alloc(sizeof(int32_t) * n);
    keys_out.alloc(sizeof(uint32_t) * n);
    vals_out.alloc(sizeof(int32_t) * n);
    k_sample_j<<<grid_for(n), BS, 0, s>>>(pix, cidx.as<int32_t>(), n, (uint32_t)n_obs,
                                          p->j.as<int32_t>(), keys.as<uint32_t>(),
                                          vals.as<int32_t>());
    unsigned end_bit = 1;
    while (end_bit < 32 && ((uint64_t)1 << end_bit) <= (uint64_t)n_obs) ++end_bit;
    tb = 0;
    MM_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys.as<uint32_t>(), keys_out.as<uint32_t>(),
                                     vals.as<int32_t>(), vals_out.as<int32_t>(), (size_t)n, 0u,
                                     end_bit, s));
    tmp.alloc(tb + 16);
    MM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tb, keys.as<uint32_t>(), keys_out.as<uint32_t>(),
                                     vals.as<int32_t>(), vals_out.as<int32_t>(), (size_t)n, 0u,
                                     end_bit, s));
    MM_HIP(hipStreamSynchronize(s));
    p->n_valid = nv;
    keys.release();
    keys_out.release();
    vals.release();
    p->perm = std::move(vals_out);  // first n_valid entries are the permutation

    // weights in time order and in pixel-sorted order; the FP64 form also
    // keeps the angles, from which its single-column P and P^T form the
    // weights on the fly (8 bytes per sample read instead of 16).  An
    // intensity-only pointing has unit weights and keeps neither.
    const bool f32 = p->prec == MM_F32;
    if (p->nc == 1) {
        std::vector<int32_t> hoff1(n_obs + 1);
        MM_HIP(hipMemcpyAsync(hoff1.data(), p->off.ptr, sizeof(int32_t) * (n_obs + 1),
                              hipMemcpyDeviceToHost, s));
        MM_HIP(hipStreamSynchronize(s));
        int32_t mx1 = 0;
        for (int32_t c = 0; c < n_obs; ++c) mx1 = std::max(mx1, hoff1[c + 1] - hoff1[c]);
        p->max_seg = mx1;
        return;
    }
    if (!f32) {
        p->psi.alloc(sizeof(double) * n);
        MM_HIP(hipMemcpyAsync(p->psi.ptr, psi, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    const size_t wsz = f32 ? sizeof(float2) : sizeof(double2);
    p->w.alloc(wsz * n);
    p->ws.alloc(wsz * (nv > 0 ? nv : 1));
    if (f32) {
        k_weights<float2><<<grid_for(n), BS, 0, s>>>(psi, n, p->w.as<float2>());
        if (nv) k_gather_w<float2><<<grid_for(nv), BS, 0, s>>>(p->perm.as<int32_t>(),
                                                              p->w.as<float2>(), nv,
                                                              p->ws.as<float2>());
    } else {
        k_weights<double2><<<grid_for(n), BS, 0, s>>>(psi, n, p->w.as<double2>());
        if (nv) k_gather_w<double2><<<grid_for(nv), BS, 0, s>>>(p->perm.as<int32_t>(),
                                                                p->w.as<double2>(), nv,
                                                                p->ws.as<double2>());
    }
    MM_HIP(hipGetLastError());

    // longest segment (used to pick the P^T launch shape)
    std::vector<int32_t> hoff(n_obs + 1);
    MM_HIP(hipMemcpyAsync(hoff.data(), p->off.ptr, sizeof(int32_t) * (n_obs + 1),
                          hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    int32_t mx = 0;
    for (int32_t c = 0; c < n_obs; ++c) mx = std::max(mx, hoff[c + 1] - hoff[c]);
    p->max_seg = mx;
    pointing_slices_device(ctx, p, 0);
}

}  // namespace mm
