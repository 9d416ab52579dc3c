// A apply that allocates nothing, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).  Its temporaries -- the two TOD vectors between P, N^-1
// and P^T, and the largest stage scratch (P's repacked map, the sliced P^T's
// partial maps, the template filter's filtered TOD) -- live in one static
// device array per GPU, `scratch`, of NOALLOC_SCRATCH_BYTES.  Its device
// address is looked up once per device with hipGetSymbolAddress at context
// creation; host code only ever passes that address, never the array's name.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "mm_internal.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;  // 128 MiB per GPU

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;  // device -> address of that device's `scratch`

char *scratch_for(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

namespace mm {

void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return;
    void *ptr = nullptr;
    MM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    MM_CHECK(ptr != nullptr, MM_E_DEVICE, "no-alloc scratch: symbol address is null");
    g_scratch_ptr[device] = static_cast<char *>(ptr);
}

}  // namespace mm

using namespace mm;

extern "C" size_t mm_apply_A_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" mm_status mm_apply_A_noalloc(mm_ctx *ctx, const mm_pointing *p, const mm_noise *nz,
                                        int32_t nrhs, const double *x, double *y,
                                        size_t *scratch_used) {
    if (!ctx) return MM_E_INVALID;
    API_BEGIN(ctx)
    MM_CHECK(p && nz, MM_E_INVALID, "apply_A_noalloc: null pointing or noise handle");
    MM_CHECK(p->n_samp == nz->n_samp && p->prec == nz->prec, MM_E_INVALID,
             "apply_A_noalloc: pointing and noise do not match");
    MM_CHECK(x && y && x != y, MM_E_INVALID,
             "apply_A_noalloc: x and y must be distinct and non-null");
    MM_CHECK(pow2_ok(nrhs), MM_E_INVALID, "nrhs must be 1, 2, 4, 8, 16, 32 or 64");
    char *base = scratch_for(ctx->device);
    MM_CHECK(base, MM_E_DEVICE, "apply_A_noalloc: scratch not set up for this device");
    const size_t te = p->prec == MM_F32 ? sizeof(float) : sizeof(double);
    const size_t tod = round256(te * (size_t)p->n_samp * nrhs);
    size_t stage = apply_P_scratch_bytes(p, nrhs);
    stage = std::max(stage, apply_PT_scratch_bytes(p, nrhs));
    stage = std::max(stage, noise_scratch_bytes(nz, nrhs));
    const size_t need = 2 * tod + round256(stage);
    if (scratch_used) *scratch_used = need;
    MM_CHECK(need <= NOALLOC_SCRATCH_BYTES, MM_E_INVALID,
             "apply_A_noalloc: needs " + std::to_string(need) + " bytes of scratch, above the " +
                 std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte maximum (use mm_apply_A)");
    // the per-stage profiler would create events; it stays off for this call
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    try {
        void *ta = base, *tb = base + tod;
        char *st = base + 2 * tod;
        apply_P_dev(ctx, p, nrhs, x, ta, st);
        noise_apply_dev(ctx, nz, nrhs, ta, tb, st);
        apply_PT_dev(ctx, p, nrhs, tb, y, st);
    } catch (...) {
        ctx->prof.on = prof;
        throw;
    }
    ctx->prof.on = prof;
    API_END
    return MM_OK;
}
