// Pointing build: hit counts, observed-pixel selection, compact pixel ids, the
// pixel-sorted sample permutation with its CSR offsets, and the polarisation
// weights (cos 2psi, sin 2psi) of Eq. datamodel, all on the device.
//
// Integer work only apart from the weights, so every integer output is
// bit-exact and independent of scheduling: the histogram uses integer atomics
// (order does not change a sum of integers); the permutation comes from a
// stable LSD radix sort of (pixel, time).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "mm_internal.h"

namespace mm {
namespace {

constexpr int BS = 256;

__global__ void k_validate(const int32_t *__restrict__ pix, const double *__restrict__ psi,
                           int64_t n, int32_t npt, int *__restrict__ flags) {
    int bad_pix = 0, bad_psi = 0;
    for (int64_t t = blockIdx.x * (int64_t)BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
        int32_t p = pix[t];
        bad_pix |= (p < -1 || p >= npt);
        bad_psi |= !isfinite(psi[t]);
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
        sincos(2.0 * psi[t], &s, &c);
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

int grid_for(int64_t n, int max_blocks = 8192) {
    int64_t g = (n + BS - 1) / BS;
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

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

    // weights in time order and in pixel-sorted order
    const bool f32 = p->prec == MM_F32;
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
}

}  // namespace mm
