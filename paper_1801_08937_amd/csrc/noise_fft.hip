// N^-1 by FFT (overlap-save per stationary interval).  Placeholder until the
// LDS-resident FFT kernel lands: reports itself unsupported so AUTO picks the
// direct band.
#include "mm_internal.h"

namespace mm {

bool noise_fft_supported(int half_bw, int64_t min_len) {
    (void)half_bw;
    (void)min_len;
    return false;
}

void noise_fft_prepare(mm_ctx *ctx, mm_noise *nz) {
    (void)ctx;
    (void)nz;
    throw Error(MM_E_INVALID, "FFT noise method not available");
}

void noise_fft_apply_dev(mm_ctx *ctx, const mm_noise *nz, int nrhs, const void *y, void *z) {
    (void)ctx; (void)nz; (void)nrhs; (void)y; (void)z;
    throw Error(MM_E_INVALID, "FFT noise method not available");
}

}  // namespace mm
